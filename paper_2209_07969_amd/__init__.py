"""MI355X phase-field fracture: Python binding of the HIP library.

Argument marshalling only (ctypes).  Every numerical step runs in the HIP
kernels of ``libphasefield.so``; this module has no CPU fallback and raises
if the library is missing or no HIP device is present.  PyTorch is used for
the device, its current stream and device tensors passed to the operator
entry points.

The C ABI is declared in ``include/phasefield.h`` (2-D solver and operators)
and ``include/phasefield3d.h`` (3-D hexahedral operators).
"""
from __future__ import annotations

import ctypes
import os
from ctypes import (CFUNCTYPE, POINTER, c_double, c_int8, c_int32, c_int64, c_size_t, c_uint8,
                    c_void_p)

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libphasefield.so")

ST, S1, S2, S3 = 0, 1, 2, 3
FP64, MIXED = 0, 1
SPLIT_VD, SPLIT_SPECTRAL = 0, 1

EXPORTED = [
    "pf_default_opts", "pf_create", "pf_destroy", "pf_set_dirichlet_u", "pf_set_dirichlet_d",
    "pf_load_step", "pf_staggered_iterate", "pf_commit_step", "pf_reaction_force",
    "pf_get_state", "pf_set_state", "pf_status_string", "pf_last_error", "pf_free_dofs",
    "pf_op_internal_force", "pf_op_tangent_apply", "pf_op_phase_apply", "pf_op_qp_update",
    "pf_op_predictor", "pf_set_profiling", "pf_kernel_time", "pf_batch_create", "pf_batch_set_workers",
    "pf_batch_load_step", "pf_batch_destroy", "pf_autotune", "pf_set_allocator",
    "pf_batch_set_shared_launches", "pf_tangent_apply_noalloc",
]
EXPORTED_3D = [
    "pf3d_op_internal_force", "pf3d_op_tangent_apply", "pf3d_op_phase_apply",
    "pf3d_op_qp_update", "pf3d_op_predictor", "pf3d_op_tangent_diag", "pf3d_op_phase_diag",
    "pf3d_op_phase_rhs", "pf3d_op_phase_coef", "pf3d_create", "pf3d_destroy",
    "pf3d_set_dirichlet_u", "pf3d_set_dirichlet_d", "pf3d_load_step", "pf3d_reaction_force",
    "pf3d_get_state", "pf3d_set_state",
]


ALLOC_FN = CFUNCTYPE(c_void_p, c_size_t, c_void_p)
RELEASE_FN = CFUNCTYPE(None, c_void_p, c_void_p)


class MeshDesc(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("lx", c_double), ("ly", c_double),
                ("elem_active", c_void_p)]


class Mesh3Desc(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("nz", c_int32), ("lx", c_double),
                ("ly", c_double), ("lz", c_double)]


class MaterialDesc(ctypes.Structure):
    _fields_ = [("E", c_double), ("nu", c_double), ("Gc", c_double), ("l", c_double),
                ("eta", c_double), ("split", c_int32)]


class SolverOpts(ctypes.Structure):
    _fields_ = [("scheme", c_int32), ("precision", c_int32), ("precond", c_int32),
                ("cheb_degree", c_int32), ("tol_stag", c_double), ("tol_pcg", c_double),
                ("tol_newton", c_double), ("tol_inner", c_double), ("max_stag", c_int32),
                ("max_newton", c_int32), ("max_cg", c_int32), ("cg_check", c_int32),
                ("psi_crit", c_double), ("d_gate", c_double), ("trial_floor", c_double),
                ("march_rows", c_int32), ("cg_kernels", c_int32),
                ("cheb_ratio", c_double), ("trial_operator", c_int32),
                ("trial_update", c_int32), ("tol_ir", c_double), ("phase_model", c_int32),
                ("guess_vectors", c_int32)]


class StepStats(ctypes.Structure):
    _fields_ = [("n_stag", c_int32), ("n_newton", c_int32), ("n_trial", c_int32),
                ("n_dsolve", c_int32), ("n_cg_u", c_int64), ("n_cg_d", c_int64),
                ("n_cg_trial", c_int64), ("gated_max", c_int64), ("floor_hits", c_int64),
                ("r_stag", c_double), ("force", c_double * 2), ("time_ms", c_double),
                ("dof_updates", c_double), ("converged", c_int32),
                ("cg_not_converged", c_int32), ("time_u_ms", c_double),
                ("time_d_ms", c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["force"] = (self.force[0], self.force[1])
        return d


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libphasefield.so and declare its signatures (no device needed)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"HIP library not built: {path} is missing (run __graft_entry__.build())")
    # PyTorch ships its own HIP runtime (same soname as the system one).  Load
    # it first so that the library binds to the runtime already in the
    # process instead of pulling in a second HIP/HSA runtime.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    P = c_void_p
    dp = POINTER(c_double)
    lib.pf_default_opts.argtypes = [POINTER(SolverOpts)]
    lib.pf_default_opts.restype = None
    lib.pf_create.argtypes = [POINTER(MeshDesc), POINTER(MaterialDesc), POINTER(SolverOpts), P,
                              POINTER(P)]
    lib.pf_destroy.argtypes = [P]
    lib.pf_set_dirichlet_u.argtypes = [P, c_int32, c_int64, POINTER(c_int64), POINTER(c_int8), dp]
    lib.pf_set_dirichlet_d.argtypes = [P, c_int64, POINTER(c_int64), dp]
    lib.pf_load_step.argtypes = [P, c_double, POINTER(StepStats)]
    lib.pf_staggered_iterate.argtypes = [P, c_double, POINTER(StepStats)]
    lib.pf_commit_step.argtypes = [P]
    lib.pf_reaction_force.argtypes = [P, c_int32, dp]
    lib.pf_get_state.argtypes = [P, dp, dp, dp]
    lib.pf_set_state.argtypes = [P, dp, dp, dp]
    lib.pf_status_string.argtypes = [c_int32]
    lib.pf_status_string.restype = ctypes.c_char_p
    lib.pf_last_error.argtypes = [P]
    lib.pf_last_error.restype = ctypes.c_char_p
    lib.pf_free_dofs.argtypes = [P, POINTER(c_int64), POINTER(c_int64)]
    lib.pf_op_internal_force.argtypes = [P, P, P, P]
    lib.pf_op_tangent_apply.argtypes = [P, P, P, P, P]
    lib.pf_op_phase_apply.argtypes = [P, P, P, P]
    lib.pf_op_qp_update.argtypes = [P, c_int32, P, P, P, P, P, P, POINTER(c_int64)]
    lib.pf_op_predictor.argtypes = [P, P, P, P, P, P, P]
    lib.pf_set_profiling.argtypes = [P, c_int32]
    lib.pf_batch_create.argtypes = [c_int32, POINTER(P), POINTER(P)]
    lib.pf_batch_set_workers.argtypes = [P, c_int32]
    lib.pf_batch_load_step.argtypes = [P, POINTER(c_double), POINTER(StepStats)]
    lib.pf_batch_destroy.argtypes = [P]
    lib.pf_batch_set_shared_launches.argtypes = [P, c_int32]
    lib.pf_autotune.argtypes = [P, c_int32, POINTER(c_int32)]
    lib.pf_set_allocator.argtypes = [P, ALLOC_FN, RELEASE_FN, P]
    lib.pf_kernel_time.argtypes = [P, c_int32, POINTER(c_int64), POINTER(c_double),
                                   POINTER(c_int64)]
    lib.pf_tangent_apply_noalloc.argtypes = [POINTER(MeshDesc), POINTER(MaterialDesc), P, P, P,
                                             P, P]
    M3, MT = POINTER(Mesh3Desc), POINTER(MaterialDesc)
    lib.pf3d_op_internal_force.argtypes = [M3, MT, P, P, P, P]
    lib.pf3d_op_tangent_apply.argtypes = [M3, MT, P, P, P, P, P]
    lib.pf3d_op_phase_apply.argtypes = [M3, MT, P, P, P, P]
    lib.pf3d_op_qp_update.argtypes = [M3, MT, c_int32, c_double, c_double, P, P, P, P, P, P, P]
    lib.pf3d_op_predictor.argtypes = [M3, MT, P, P, P, P, P, P, P]
    lib.pf3d_op_tangent_diag.argtypes = [M3, MT, P, P, P, P]
    lib.pf3d_op_phase_diag.argtypes = [M3, MT, P, P, P]
    lib.pf3d_op_phase_rhs.argtypes = [M3, P, P, P]
    lib.pf3d_op_phase_coef.argtypes = [M3, MT, c_int32, c_double, c_int32, P, P, P, P, P, P]
    lib.pf3d_create.argtypes = [M3, MT, POINTER(SolverOpts), P, POINTER(P)]
    lib.pf3d_destroy.argtypes = [P]
    lib.pf3d_set_dirichlet_u.argtypes = [P, c_int32, c_int64, POINTER(c_int64), POINTER(c_int8),
                                         dp]
    lib.pf3d_set_dirichlet_d.argtypes = [P, c_int64, POINTER(c_int64), dp]
    lib.pf3d_load_step.argtypes = [P, c_double, POINTER(StepStats)]
    lib.pf3d_reaction_force.argtypes = [P, c_int32, dp]
    lib.pf3d_get_state.argtypes = [P, dp, dp, dp]
    lib.pf3d_set_state.argtypes = [P, dp, dp, dp]
    for name in EXPORTED + EXPORTED_3D:
        if name != "pf_default_opts" and name not in ("pf_status_string", "pf_last_error"):
            getattr(lib, name).restype = c_int32
    _lib = lib
    return lib


def require_device():
    """Raise unless the HIP library loads and a HIP device is visible."""
    load_library()
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device visible: the phase-field library has no CPU path")


class PhaseFieldError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{status}: {msg}")
        self.status = status


STATUS_NOT_CONVERGED = 5


def _ptr(a, ctype):
    return a.ctypes.data_as(POINTER(ctype))


def _dev_arg(t, dtype, count, device, name):
    """Pointer to tensor t after checking what the C ABI cannot: its dtype,
    that it holds at least `count` elements (the kernels read or write that
    many), that it is contiguous and resident on the context's device."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch.Tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name}: expected dtype {dtype}, got {t.dtype}")
    if t.numel() < count:
        raise ValueError(f"{name}: needs {count} elements, got {t.numel()}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous tensor")
    if not t.is_cuda:
        raise ValueError(f"{name}: expected a device tensor")
    if t.device.index != device:
        raise ValueError(f"{name}: tensor is on device {t.device.index}, the context on {device}")
    return c_void_p(t.data_ptr())


def default_opts() -> SolverOpts:
    o = SolverOpts()
    load_library().pf_default_opts(ctypes.byref(o))
    return o


class Context:
    """One fracture problem on the current HIP device.

    ``problem`` is any object with the attributes of ``workloads.Problem``
    (nx, ny, lx, ly, material, dir_u, dir_d_nodes, dir_d_values, elem_active,
    tolerances).  Options not given are taken from the problem, then from the
    library defaults.
    """

    def __init__(self, problem, scheme=ST, precision=FP64, stream=None, **overrides):
        require_device()
        import torch
        self.lib = load_library()
        self.p = problem
        p = problem
        self._mask = None
        mesh = MeshDesc(int(p.nx), int(p.ny), float(p.lx), float(p.ly), None)
        if getattr(p, "elem_active", None) is not None:
            self._mask = np.ascontiguousarray(p.elem_active, dtype=np.uint8)
            mesh.elem_active = self._mask.ctypes.data_as(c_void_p)
        m = p.material
        mat = MaterialDesc(m.E, m.nu, m.Gc, m.l, m.eta, int(m.split))
        o = default_opts()
        o.scheme = int(scheme)
        o.precision = int(precision)
        for name in ("tol_stag", "tol_pcg", "tol_newton", "max_stag", "max_newton",
                     "psi_crit", "d_gate", "trial_floor", "trial_operator", "trial_update",
                     "phase_model", "tol_ir"):
            if hasattr(p, name):
                setattr(o, name, getattr(p, name))
        for k, v in overrides.items():
            setattr(o, k, v)
        self.opts = o
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.stream = stream
        h = c_void_p()
        st = self.lib.pf_create(ctypes.byref(mesh), ctypes.byref(mat), ctypes.byref(o),
                                c_void_p(stream), ctypes.byref(h))
        if st != 0:
            raise PhaseFieldError(st, "pf_create failed: " +
                                  self.lib.pf_status_string(st).decode())
        self.h = h
        self.device = torch.cuda.current_device()
        self.N = (p.nx + 1) * (p.ny + 1)
        self.E = p.nx * p.ny
        for gi, grp in enumerate(p.dir_u):
            self.set_dirichlet_u(gi, grp.nodes, grp.comps, grp.values)
        self.set_dirichlet_d(p.dir_d_nodes, p.dir_d_values)

    # ----------------------------------------------------------- helpers
    def _check(self, st, what):
        if st != 0:
            msg = self.lib.pf_last_error(self.h).decode()
            raise PhaseFieldError(st, f"{what}: {self.lib.pf_status_string(st).decode()} ({msg})")

    def close(self):
        if getattr(self, "h", None):
            self.lib.pf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --------------------------------------------------------------- API
    def set_dirichlet_u(self, group, nodes, comps, values):
        n = np.ascontiguousarray(nodes, dtype=np.int64)
        c = np.ascontiguousarray(comps, dtype=np.int8)
        v = np.ascontiguousarray(values, dtype=np.float64)
        self._check(self.lib.pf_set_dirichlet_u(self.h, group, n.size, _ptr(n, c_int64),
                                                _ptr(c, c_int8), _ptr(v, c_double)),
                    "pf_set_dirichlet_u")

    def set_dirichlet_d(self, nodes, values):
        n = np.ascontiguousarray(nodes, dtype=np.int64)
        v = np.ascontiguousarray(values, dtype=np.float64)
        self._check(self.lib.pf_set_dirichlet_d(self.h, n.size, _ptr(n, c_int64),
                                                _ptr(v, c_double)), "pf_set_dirichlet_d")

    def load_step(self, lam, allow_not_converged=True):
        st = StepStats()
        s = self.lib.pf_load_step(self.h, float(lam), ctypes.byref(st))
        if s != 0 and not (allow_not_converged and s == STATUS_NOT_CONVERGED):
            self._check(s, "pf_load_step")
        return st.as_dict()

    def staggered_iterate(self, lam):
        st = StepStats()
        self._check(self.lib.pf_staggered_iterate(self.h, float(lam), ctypes.byref(st)),
                    "pf_staggered_iterate")
        return st.as_dict()

    def commit_step(self):
        self._check(self.lib.pf_commit_step(self.h), "pf_commit_step")

    def reaction_force(self, group=1):
        f = np.zeros(2)
        self._check(self.lib.pf_reaction_force(self.h, group, _ptr(f, c_double)),
                    "pf_reaction_force")
        return f

    def get_state(self):
        u = np.zeros(2 * self.N)
        d = np.zeros(self.N)
        H = np.zeros(4 * self.E)
        self._check(self.lib.pf_get_state(self.h, _ptr(u, c_double), _ptr(d, c_double),
                                          _ptr(H, c_double)), "pf_get_state")
        return u.reshape(2, self.N), d, H.reshape(4, self.E)

    def set_state(self, u=None, d=None, H=None):
        def arr(x, n):
            if x is None:
                return None, None
            a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1))
            if a.size != n:
                raise ValueError("state array has the wrong size")
            return a, _ptr(a, c_double)
        ua, up = arr(u, 2 * self.N)
        da, dpp = arr(d, self.N)
        Ha, Hp = arr(H, 4 * self.E)
        self._check(self.lib.pf_set_state(self.h, up, dpp, Hp), "pf_set_state")

    def free_dofs(self):
        a, b = c_int64(), c_int64()
        self._check(self.lib.pf_free_dofs(self.h, ctypes.byref(a), ctypes.byref(b)),
                    "pf_free_dofs")
        return a.value, b.value

    def autotune(self, reps=20):
        """Pick the fastest work-item height for this mesh; returns it."""
        ch = c_int32()
        self._check(self.lib.pf_autotune(self.h, int(reps), ctypes.byref(ch)), "pf_autotune")
        return ch.value

    def use_torch_allocator(self):
        """Move the context's device buffers into PyTorch's caching allocator
        (blocks tied to the context's stream); pf_destroy returns them."""
        import torch
        dev = torch.cuda.current_device()
        stream = int(self.stream or 0)

        def alloc(nbytes, _user):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), dev, stream)
            except RuntimeError:
                return None

        def release(ptr, _user):
            torch.cuda.caching_allocator_delete(ptr)

        cbs = (ALLOC_FN(alloc), RELEASE_FN(release))
        self._check(self.lib.pf_set_allocator(self.h, cbs[0], cbs[1], None), "pf_set_allocator")
        self._alloc_cbs = cbs      # must outlive the buffers

    def use_default_allocator(self):
        """Move the buffers back to hipMalloc memory."""
        self._check(self.lib.pf_set_allocator(self.h, ALLOC_FN(), RELEASE_FN(), None),
                    "pf_set_allocator")
        self._alloc_cbs = None

    def set_profiling(self, enable=True):
        self._check(self.lib.pf_set_profiling(self.h, 1 if enable else 0), "pf_set_profiling")

    def kernel_time(self, kernel):
        """(sampled launches, total ms, nodes per launch) of a CG kernel."""
        n, ms, nodes = c_int64(), c_double(), c_int64()
        self._check(self.lib.pf_kernel_time(self.h, int(kernel), ctypes.byref(n),
                                            ctypes.byref(ms), ctypes.byref(nodes)),
                    "pf_kernel_time")
        return n.value, ms.value, nodes.value

    # ------------------------------------------------- operator entries
    # Device tensors in the layouts of include/phasefield.h: displacement
    # fields [2N] (x plane, then y plane), nodal fields [N], quadrature-point
    # fields [4E] (plane q holds point q of every element), flags [E] (uint8).
    def _nodal(self, t, name, comps=1):
        import torch
        return _dev_arg(t, torch.float64, comps * self.N, self.device, name)

    def _qp(self, t, name):
        import torch
        return _dev_arg(t, torch.float64, 4 * self.E, self.device, name)

    def _flags(self, t, name):
        import torch
        return _dev_arg(t, torch.uint8, self.E, self.device, name)

    def op_internal_force(self, u, d, R):
        self._check(self.lib.pf_op_internal_force(self.h, self._nodal(u, "u", 2),
                                                  self._nodal(d, "d"), self._nodal(R, "R", 2)),
                    "pf_op_internal_force")

    def op_tangent_apply(self, u, d, p, q):
        self._check(self.lib.pf_op_tangent_apply(self.h, self._nodal(u, "u", 2), self._nodal(d, "d"),
                                                 self._nodal(p, "p", 2), self._nodal(q, "q", 2)),
                    "pf_op_tangent_apply")

    def op_phase_apply(self, coef, p, q):
        self._check(self.lib.pf_op_phase_apply(self.h, self._qp(coef, "coef"), self._nodal(p, "p"),
                                               self._nodal(q, "q")), "pf_op_phase_apply")

    def op_qp_update(self, scheme, u, d, H_prev, H, psi_s, flags):
        n = c_int64()
        self._check(self.lib.pf_op_qp_update(self.h, int(scheme), self._nodal(u, "u", 2),
                                             self._nodal(d, "d"), self._qp(H_prev, "H_prev"),
                                             self._qp(H, "H"), self._qp(psi_s, "psi_s"),
                                             self._flags(flags, "flags"), ctypes.byref(n)),
                    "pf_op_qp_update")
        return n.value

    def op_predictor(self, d, dd, H, psi_s, flags, Hhat):
        self._check(self.lib.pf_op_predictor(self.h, self._nodal(d, "d"), self._nodal(dd, "dd"),
                                             self._qp(H, "H"), self._qp(psi_s, "psi_s"),
                                             self._flags(flags, "flags"), self._qp(Hhat, "Hhat")),
                    "pf_op_predictor")


NOALLOC_MAX_ELEMENTS = 16 * 1024 * 1024


def tangent_apply_noalloc(problem, u, d, p, q, elem_active=None, stream=None):
    """pf_tangent_apply_noalloc: q = K_t(u; d) p without a context and
    without device allocation.  problem: nx, ny, lx, ly and material as for
    Context; u, p, q [2N] and d [N] float64 device tensors on the current
    device; elem_active: None or a uint8 device tensor [nx*ny]; stream: a
    hipStream_t handle (None = torch's current stream)."""
    import torch
    require_device()
    lib = load_library()
    dev = torch.cuda.current_device()
    N = (problem.nx + 1) * (problem.ny + 1)
    mask = None if elem_active is None else _dev_arg(elem_active, torch.uint8,
                                                      problem.nx * problem.ny, dev,
                                                      "elem_active").value
    mesh = MeshDesc(int(problem.nx), int(problem.ny), float(problem.lx), float(problem.ly), mask)
    m = problem.material
    mat = MaterialDesc(m.E, m.nu, m.Gc, m.l, m.eta, int(m.split))
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    st = lib.pf_tangent_apply_noalloc(
        ctypes.byref(mesh), ctypes.byref(mat), _dev_arg(u, torch.float64, 2 * N, dev, "u"),
        _dev_arg(d, torch.float64, N, dev, "d"), _dev_arg(p, torch.float64, 2 * N, dev, "p"),
        _dev_arg(q, torch.float64, 2 * N, dev, "q"), c_void_p(stream))
    if st != 0:
        raise PhaseFieldError(st, "pf_tangent_apply_noalloc: " +
                              lib.pf_status_string(st).decode())


class Hex3DOps:
    """The 3-D operator entry points (include/phasefield3d.h) on the box mesh
    of ``problem`` (any object with nx, ny, nz, lx, ly, lz and a material;
    either split).  Device tensors in the header's layouts:
    displacement fields [3N] (x, y, z planes), nodal fields [N],
    quadrature-point fields [8E] (plane q holds point q of every element),
    flags [E] (int16 tensors holding the uint16 flag words).  Kernels go to
    torch's current stream."""

    def __init__(self, problem):
        require_device()
        import torch
        self.lib = load_library()
        p = problem
        self.mesh = Mesh3Desc(int(p.nx), int(p.ny), int(p.nz), float(p.lx), float(p.ly),
                              float(p.lz))
        m = p.material
        self.mat = MaterialDesc(m.E, m.nu, m.Gc, m.l, m.eta, int(m.split))
        self.device = torch.cuda.current_device()
        self.N = (p.nx + 1) * (p.ny + 1) * (p.nz + 1)
        self.E = p.nx * p.ny * p.nz

    def _arg(self, t, count, name, dtype=None):
        import torch
        return _dev_arg(t, torch.float64 if dtype is None else dtype, count, self.device, name)

    def _stream(self):
        import torch
        return c_void_p(torch.cuda.current_stream().cuda_stream)

    def _check(self, st, what):
        if st != 0:
            raise PhaseFieldError(st, f"{what}: {self.lib.pf_status_string(st).decode()}")

    def internal_force(self, u, d, R):
        N = self.N
        self._check(self.lib.pf3d_op_internal_force(
            ctypes.byref(self.mesh), ctypes.byref(self.mat), self._arg(u, 3 * N, "u"),
            self._arg(d, N, "d"), self._arg(R, 3 * N, "R"), self._stream()),
            "pf3d_op_internal_force")

    def tangent_apply(self, u, d, p, q):
        N = self.N
        self._check(self.lib.pf3d_op_tangent_apply(
            ctypes.byref(self.mesh), ctypes.byref(self.mat), self._arg(u, 3 * N, "u"),
            self._arg(d, N, "d"), self._arg(p, 3 * N, "p"), self._arg(q, 3 * N, "q"),
            self._stream()), "pf3d_op_tangent_apply")

    def phase_apply(self, coef, p, q):
        self._check(self.lib.pf3d_op_phase_apply(
            ctypes.byref(self.mesh), ctypes.byref(self.mat), self._arg(coef, 8 * self.E, "coef"),
            self._arg(p, self.N, "p"), self._arg(q, self.N, "q"), self._stream()),
            "pf3d_op_phase_apply")

    def qp_update(self, scheme, psi_crit, d_gate, u, d, H_prev, H, psi_s, flags):
        import torch
        N, E8 = self.N, 8 * self.E
        self._check(self.lib.pf3d_op_qp_update(
            ctypes.byref(self.mesh), ctypes.byref(self.mat), int(scheme), float(psi_crit),
            float(d_gate), self._arg(u, 3 * N, "u"), self._arg(d, N, "d"),
            self._arg(H_prev, E8, "H_prev"), self._arg(H, E8, "H"), self._arg(psi_s, E8, "psi_s"),
            self._arg(flags, self.E, "flags", torch.int16), self._stream()),
            "pf3d_op_qp_update")

    def predictor(self, d, dd, H, psi_s, flags, Hhat):
        import torch
        N, E8 = self.N, 8 * self.E
        self._check(self.lib.pf3d_op_predictor(
            ctypes.byref(self.mesh), ctypes.byref(self.mat), self._arg(d, N, "d"),
            self._arg(dd, N, "dd"), self._arg(H, E8, "H"), self._arg(psi_s, E8, "psi_s"),
            self._arg(flags, self.E, "flags", torch.int16), self._arg(Hhat, E8, "Hhat"),
            self._stream()), "pf3d_op_predictor")

    def tangent_diag(self, u, d, D):
        N = self.N
        self._check(self.lib.pf3d_op_tangent_diag(
            ctypes.byref(self.mesh), ctypes.byref(self.mat), self._arg(u, 3 * N, "u"),
            self._arg(d, N, "d"), self._arg(D, 3 * N, "D"), self._stream()),
            "pf3d_op_tangent_diag")

    def phase_diag(self, coef, D):
        self._check(self.lib.pf3d_op_phase_diag(
            ctypes.byref(self.mesh), ctypes.byref(self.mat), self._arg(coef, 8 * self.E, "coef"),
            self._arg(D, self.N, "D"), self._stream()), "pf3d_op_phase_diag")

    def phase_rhs(self, H, b):
        self._check(self.lib.pf3d_op_phase_rhs(
            ctypes.byref(self.mesh), self._arg(H, 8 * self.E, "H"), self._arg(b, self.N, "b"),
            self._stream()), "pf3d_op_phase_rhs")

    def phase_coef(self, H, coef, trial=None):
        """AT2 coefficient, or with trial = (theta, floor, psi_s, flags, d)
        the trial block's."""
        import torch
        E8 = 8 * self.E
        if trial is None:
            args = (0, 0.0, 0, None, None, None)
        else:
            theta, floor, psi_s, flags, d = trial
            args = (1, float(theta), int(floor), self._arg(psi_s, E8, "psi_s"),
                    self._arg(flags, self.E, "flags", torch.int16), self._arg(d, self.N, "d"))
        self._check(self.lib.pf3d_op_phase_coef(
            ctypes.byref(self.mesh), ctypes.byref(self.mat), args[0], args[1], args[2],
            self._arg(H, E8, "H"), args[3], args[4], args[5], self._arg(coef, E8, "coef"),
            self._stream()), "pf3d_op_phase_coef")


class Hex3DContext:
    """A 3-D load history on a box of trilinear hexahedra (pf3d_create):
    ``problem`` has the attributes of ``workloads.Problem3D``.  FP64 with
    Jacobi PCG, AT2 with the history field; ``scheme`` ST or S1/S2/S3 with
    the floored trial block."""

    def __init__(self, problem, scheme=ST, stream=None, **overrides):
        require_device()
        import torch
        self.lib = load_library()
        p = problem
        self.p = p
        mesh = Mesh3Desc(int(p.nx), int(p.ny), int(p.nz), float(p.lx), float(p.ly), float(p.lz))
        m = p.material
        mat = MaterialDesc(m.E, m.nu, m.Gc, m.l, m.eta, int(m.split))
        o = default_opts()
        o.scheme = int(scheme)
        for name in ("tol_stag", "tol_pcg", "tol_newton", "max_stag", "max_newton",
                     "psi_crit", "d_gate", "trial_floor"):
            if hasattr(p, name):
                setattr(o, name, getattr(p, name))
        for k, v in overrides.items():
            setattr(o, k, v)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        h = c_void_p()
        st = self.lib.pf3d_create(ctypes.byref(mesh), ctypes.byref(mat), ctypes.byref(o),
                                  c_void_p(stream), ctypes.byref(h))
        if st != 0:
            raise PhaseFieldError(st, "pf3d_create failed: " +
                                  self.lib.pf_status_string(st).decode())
        self.h = h
        self.N = (p.nx + 1) * (p.ny + 1) * (p.nz + 1)
        self.E = p.nx * p.ny * p.nz
        for gi, grp in enumerate(p.dir_u):
            n = np.ascontiguousarray(grp.nodes, dtype=np.int64)
            c = np.ascontiguousarray(grp.comps, dtype=np.int8)
            v = np.ascontiguousarray(grp.values, dtype=np.float64)
            self._check(self.lib.pf3d_set_dirichlet_u(self.h, gi, n.size, _ptr(n, c_int64),
                                                      _ptr(c, c_int8), _ptr(v, c_double)),
                        "pf3d_set_dirichlet_u")
        n = np.ascontiguousarray(p.dir_d_nodes, dtype=np.int64)
        v = np.ascontiguousarray(p.dir_d_values, dtype=np.float64)
        self._check(self.lib.pf3d_set_dirichlet_d(self.h, n.size, _ptr(n, c_int64),
                                                  _ptr(v, c_double)), "pf3d_set_dirichlet_d")

    def _check(self, st, what):
        if st != 0:
            raise PhaseFieldError(st, f"{what}: {self.lib.pf_status_string(st).decode()}")

    def load_step(self, lam, allow_not_converged=True):
        st = StepStats()
        s = self.lib.pf3d_load_step(self.h, float(lam), ctypes.byref(st))
        if s != 0 and not (allow_not_converged and s == STATUS_NOT_CONVERGED):
            self._check(s, "pf3d_load_step")
        return st.as_dict()

    def reaction_force(self, group=1):
        f = np.zeros(3)
        self._check(self.lib.pf3d_reaction_force(self.h, group, _ptr(f, c_double)),
                    "pf3d_reaction_force")
        return f

    def get_state(self):
        u, d, H = np.zeros(3 * self.N), np.zeros(self.N), np.zeros(8 * self.E)
        self._check(self.lib.pf3d_get_state(self.h, _ptr(u, c_double), _ptr(d, c_double),
                                            _ptr(H, c_double)), "pf3d_get_state")
        return u.reshape(3, self.N), d, H.reshape(8, self.E)

    def set_state(self, u=None, d=None, H=None):
        def arr(x, n):
            if x is None:
                return None, None
            a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1))
            if a.size != n:
                raise ValueError("state array has the wrong size")
            return a, _ptr(a, c_double)
        ua, up = arr(u, 3 * self.N)
        da, dpp = arr(d, self.N)
        Ha, Hp = arr(H, 8 * self.E)
        self._check(self.lib.pf3d_set_state(self.h, up, dpp, Hp), "pf3d_set_state")

    def close(self):
        if getattr(self, "h", None):
            self.lib.pf3d_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Several contexts advanced together (each should own a HIP stream, e.g.
    Context(..., stream=torch.cuda.Stream().cuda_stream)).  shared=True runs
    the members' FP32 Jacobi CG solves through shared launches; False runs the
    members concurrently on their streams from `workers` host threads."""

    def __init__(self, contexts, workers=4, shared=True):
        self.lib = load_library()
        self.members = list(contexts)
        arr = (c_void_p * len(self.members))(*[c.h for c in self.members])
        h = c_void_p()
        st = self.lib.pf_batch_create(len(self.members), arr, ctypes.byref(h))
        if st != 0:
            raise PhaseFieldError(st, "pf_batch_create failed")
        self.h = h
        st = self.lib.pf_batch_set_workers(h, int(workers))
        if st != 0:
            raise PhaseFieldError(st, "pf_batch_set_workers failed")
        st = self.lib.pf_batch_set_shared_launches(h, 1 if shared else 0)
        if st != 0:
            raise PhaseFieldError(st, "pf_batch_set_shared_launches failed")

    def load_step(self, load_factors, allow_not_converged=True):
        if any(not getattr(c, "h", None) for c in self.members):
            raise RuntimeError("a member context was closed before the batch")
        n = len(self.members)
        lam = np.ascontiguousarray(load_factors, dtype=np.float64)
        if lam.size != n:
            raise ValueError("one load factor per member")
        stats = (StepStats * n)()
        s = self.lib.pf_batch_load_step(self.h, _ptr(lam, c_double), stats)
        if s != 0 and not (allow_not_converged and s == STATUS_NOT_CONVERGED):
            raise PhaseFieldError(s, "pf_batch_load_step: " + self.lib.pf_status_string(s).decode())
        return [stats[i].as_dict() for i in range(n)]

    def close(self):
        if getattr(self, "h", None):
            self.lib.pf_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


__all__ = ["Batch", "Context", "Hex3DContext", "Hex3DOps", "load_library", "require_device", "default_opts", "PhaseFieldError",
           "ST", "S1", "S2", "S3", "FP64", "MIXED", "EXPORTED"]
