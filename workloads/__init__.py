"""Synthetic phase-field fracture workloads (inputs only).

This module describes *what* is solved: a structured rectangular Q1 mesh, the
material, the Dirichlet data for the displacement u and the phase field d, and
the load history.  It holds none of the method's arithmetic (no strains, no
energies, no operators), so that the CPU oracle (``oracle/``) and the HIP path
(``paper_2209_07969_amd``) can both consume the same seeded inputs while
sharing no code that computes anything.

Conventions (shared by both sides because they are *input* conventions):

* Domain [0, lx] x [0, ly], ``nx`` x ``ny`` bilinear quadrilaterals.
* Node (i, j), 0 <= i <= nx, 0 <= j <= ny, has id ``i + j*(nx+1)``.
* Element (i, j) has id ``i + j*nx`` and corners (i,j), (i+1,j), (i+1,j+1),
  (i,j+1) in that order.
* An optional element mask (``elem_active``, uint8, length nx*ny) removes
  elements; a node is active iff it touches an active element.
* Displacement Dirichlet data is given per group: node ids, component
  (0 = x, 1 = y) and a value per unit load factor; at load factor lambda the
  prescribed value is lambda * value.  Group 0 is conventionally the fixed
  support and group 1 the loaded edge whose reaction force is reported.
* Phase-field Dirichlet data: node ids and fixed values (e.g. a notch d = 1).
* Units: N, mm, MPa; forces per unit thickness.

The concrete panels stand in for the paper's tensile, shear and L-shaped
panel experiments (Section 4.1-4.3), whose meshes are not published.
"""
from __future__ import annotations

import dataclasses
import json
from typing import List, Optional

import numpy as np

# Split identifiers
SPLIT_VD = 0          # volumetric-deviatoric (Amor) split, Section 2
SPLIT_SPECTRAL = 1    # spectral (Miehe) split, named in Section 2

# Scheme identifiers (Section 3.4, table of assumptions)
ST, S1, S2, S3 = 0, 1, 2, 3
SCHEME_NAMES = {ST: "ST", S1: "S1", S2: "S2", S3: "S3"}


@dataclasses.dataclass
class Material:
    E: float = 2.1e5      # Young's modulus [MPa]
    nu: float = 0.3       # Poisson ratio
    Gc: float = 2.7       # critical energy release rate [N/mm]
    l: float = 0.03       # regularisation length [mm]
    eta: float = 1e-6     # residual stiffness in g(d) = (1-d)^2 + eta
    split: int = SPLIT_VD


@dataclasses.dataclass
class DirichletU:
    nodes: np.ndarray     # int64 node ids
    comps: np.ndarray     # int8, 0 = x, 1 = y
    values: np.ndarray    # float64, value per unit load factor


@dataclasses.dataclass
class Problem:
    name: str
    nx: int
    ny: int
    lx: float
    ly: float
    material: Material
    dir_u: List[DirichletU]
    dir_d_nodes: np.ndarray
    dir_d_values: np.ndarray
    loads: np.ndarray                  # load factor per step
    elem_active: Optional[np.ndarray] = None   # uint8 [nx*ny] or None
    load_group: int = 1
    load_comp: int = 1                 # component whose reaction is reported
    # solver settings shared by both sides
    tol_stag: float = 1e-5
    tol_pcg: float = 1e-10
    tol_newton: float = 1e-9
    max_stag: int = 500
    max_newton: int = 25
    psi_crit: float = -1.0             # < 0 means Gc / (c_w l) with c_w = 2
    d_gate: float = 0.95
    trial_floor: float = 0.1
    trial_operator: int = 0            # 0: mass coefficient floored at theta c; 1: unfloored
    trial_update: int = 0              # 0: trial -> predict -> correct; 1: d += trial increment
    phase_model: int = 0               # 0: AT2 with history field; 1: AT1 with penalty
    tol_ir: float = 0.01               # irreversibility tolerance of the penalty (AT1)

    @property
    def n_nodes(self) -> int:
        return (self.nx + 1) * (self.ny + 1)

    @property
    def n_elems(self) -> int:
        return self.nx * self.ny

    def node_id(self, i, j):
        return np.asarray(i) + np.asarray(j) * (self.nx + 1)

    def with_steps(self, n_steps: int) -> "Problem":
        p = dataclasses.replace(self)
        du = self.loads[0] if len(self.loads) else 0.0
        p.loads = du * np.arange(1, n_steps + 1, dtype=np.float64)
        return p


def _edge_nodes(nx, ny, edge):
    if edge == "bottom":
        return np.arange(0, nx + 1, dtype=np.int64)
    if edge == "top":
        return np.arange(0, nx + 1, dtype=np.int64) + ny * (nx + 1)
    if edge == "left":
        return np.arange(0, ny + 1, dtype=np.int64) * (nx + 1)
    if edge == "right":
        return np.arange(0, ny + 1, dtype=np.int64) * (nx + 1) + nx
    raise ValueError(edge)


def _fix(nodes, comps, val=0.0):
    nodes = np.asarray(nodes, dtype=np.int64)
    out_n, out_c = [], []
    for c in comps:
        out_n.append(nodes)
        out_c.append(np.full(nodes.shape, c, dtype=np.int8))
    n = np.concatenate(out_n)
    c = np.concatenate(out_c)
    return DirichletU(n, c, np.full(n.shape, val, dtype=np.float64))


def notch_nodes(nx, ny, lx, ly, a, y0=0.5):
    """Nodes on the horizontal line y = y0*ly with x <= a (notch as d = 1)."""
    j = int(round(y0 * ny))
    if abs(j / ny - y0) > 1e-12:
        raise ValueError("notch line y0 must fall on a node row")
    i = np.arange(0, nx + 1)
    x = i * (lx / nx)
    sel = i[x <= a + 1e-12 * lx]
    return (sel + j * (nx + 1)).astype(np.int64)


def tension_panel(n=64, l=0.03, du=3e-4, steps=20, notch=0.5, Gc=2.7,
                  E=2.1e5, nu=0.3, eta=1e-6, split=SPLIT_VD,
                  name="tension") -> Problem:
    """Single-edge-notched tension panel on the unit square.

    Bottom edge: both components fixed.  Top edge: u_y = lambda, u_x free.
    Notch: nodes with y = 0.5 and x <= notch carry the Dirichlet value d = 1.
    """
    nx = ny = n
    bottom = _fix(_edge_nodes(nx, ny, "bottom"), (0, 1))
    top = DirichletU(_edge_nodes(nx, ny, "top"),
                     np.full(nx + 1, 1, dtype=np.int8),
                     np.ones(nx + 1, dtype=np.float64))
    dn = notch_nodes(nx, ny, 1.0, 1.0, notch)
    return Problem(name=name, nx=nx, ny=ny, lx=1.0, ly=1.0,
                   material=Material(E=E, nu=nu, Gc=Gc, l=l, eta=eta, split=split),
                   dir_u=[bottom, top], dir_d_nodes=dn,
                   dir_d_values=np.ones(dn.shape, dtype=np.float64),
                   loads=du * np.arange(1, steps + 1, dtype=np.float64),
                   load_group=1, load_comp=1)


def shear_panel(n=1024, l=0.004, du=1e-4, steps=150, notch=0.5,
                split=SPLIT_SPECTRAL, name="shear") -> Problem:
    """Single-edge-notched shear panel: bottom fixed, top u_x = lambda, u_y = 0."""
    nx = ny = n
    bottom = _fix(_edge_nodes(nx, ny, "bottom"), (0, 1))
    topn = _edge_nodes(nx, ny, "top")
    top = DirichletU(np.concatenate([topn, topn]),
                     np.concatenate([np.zeros(nx + 1, np.int8), np.ones(nx + 1, np.int8)]),
                     np.concatenate([np.ones(nx + 1), np.zeros(nx + 1)]))
    dn = notch_nodes(nx, ny, 1.0, 1.0, notch)
    return Problem(name=name, nx=nx, ny=ny, lx=1.0, ly=1.0,
                   material=Material(l=l, split=split),
                   dir_u=[bottom, top], dir_d_nodes=dn,
                   dir_d_values=np.ones(dn.shape),
                   loads=du * np.arange(1, steps + 1, dtype=np.float64),
                   load_group=1, load_comp=0)


def lshape_panel(n=2048, steps=200, total=1.0, name="lshape") -> Problem:
    """L-shaped panel [0,500]^2 minus the upper-right quadrant.

    All nodes on y = 0 are fixed.  The load u_y = lambda acts on the nodes of
    the arm's top face y = 250 with |x - 280| <= 4h.  Nodes within 4 l of the
    load point (280, 250) carry the Dirichlet value d = 0.
    """
    nx = ny = n
    L = 500.0
    h = L / n
    jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    xc = (ii + 0.5) * h
    yc = (jj + 0.5) * h
    active = ~((xc > 250.0) & (yc > 250.0))
    elem_active = active.astype(np.uint8).reshape(-1)
    bottom = _fix(_edge_nodes(nx, ny, "bottom"), (0, 1))
    jrow = int(round(250.0 / h))
    i = np.arange(nx + 1)
    x = i * h
    sel = i[np.abs(x - 280.0) <= 4 * h + 1e-9]
    load_nodes = (sel + jrow * (nx + 1)).astype(np.int64)
    top = DirichletU(load_nodes, np.ones(load_nodes.shape, np.int8),
                     np.ones(load_nodes.shape))
    mat = Material(E=2.585e4, nu=0.18, Gc=0.095, l=2.0, eta=1e-6, split=SPLIT_VD)
    jn, inn = np.meshgrid(np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    xn = inn * h
    yn = jn * h
    near = ((xn - 280.0) ** 2 + (yn - 250.0) ** 2 <= (4 * mat.l) ** 2).reshape(-1)
    # keep only active nodes (those touching an active element): in the masked
    # quadrant (x > 250 and y > 250 strictly) no node is active
    inside_hole = ((xn > 250.0 + 1e-9) & (yn > 250.0 + 1e-9)).reshape(-1)
    dn = np.nonzero(near & ~inside_hole)[0].astype(np.int64)
    return Problem(name=name, nx=nx, ny=ny, lx=L, ly=L, material=mat,
                   dir_u=[bottom, top], dir_d_nodes=dn,
                   dir_d_values=np.zeros(dn.shape),
                   loads=(total / steps) * np.arange(1, steps + 1, dtype=np.float64),
                   elem_active=elem_active, load_group=1, load_comp=1)


def homogeneous_bar(nx=4, ny=4, lx=1.0, ly=1.0, E=2.1e5, nu=0.3, Gc=2.7, l=0.03,
                    eta=1e-6, du=1e-3, steps=5, name="bar") -> Problem:
    """Un-notched bar on rollers: bottom u_y = 0, bottom-left u_x = 0, top u_y = lambda."""
    bottom_n = _edge_nodes(nx, ny, "bottom")
    fixed = DirichletU(np.concatenate([bottom_n, np.array([0], np.int64)]),
                       np.concatenate([np.ones(nx + 1, np.int8), np.zeros(1, np.int8)]),
                       np.zeros(nx + 2))
    top = DirichletU(_edge_nodes(nx, ny, "top"), np.ones(nx + 1, np.int8),
                     np.ones(nx + 1))
    return Problem(name=name, nx=nx, ny=ny, lx=lx, ly=ly,
                   material=Material(E=E, nu=nu, Gc=Gc, l=l, eta=eta),
                   dir_u=[fixed, top], dir_d_nodes=np.zeros(0, np.int64),
                   dir_d_values=np.zeros(0),
                   loads=du * np.arange(1, steps + 1, dtype=np.float64),
                   load_group=1, load_comp=1)


# --------------------------------------------------------------------------
# Three dimensions (Q1 hexahedra): a slab extruded from a 2-D panel, and a
# uniaxial bar
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Problem3D:
    name: str
    nx: int
    ny: int
    nz: int
    lx: float
    ly: float
    lz: float
    material: Material
    dir_u: List[DirichletU]            # comps 0, 1, 2 = x, y, z
    dir_d_nodes: np.ndarray
    dir_d_values: np.ndarray
    loads: np.ndarray
    load_group: int = 1
    load_comp: int = 1
    tol_stag: float = 1e-5
    tol_pcg: float = 1e-10
    tol_newton: float = 1e-9
    max_stag: int = 500
    max_newton: int = 25
    psi_crit: float = -1.0
    d_gate: float = 0.95
    trial_floor: float = 0.1


def slab_from_panel(p: Problem, nz: int = 1, lz: float = 0.1) -> Problem3D:
    """The 2-D panel extruded over nz element layers of total thickness lz:
    its Dirichlet data on every node layer, and u_z = 0 everywhere on both
    faces z = 0 and z = lz (with nz = 1: on every node, i.e. plane strain)."""
    P = (p.nx + 1) * (p.ny + 1)
    layers = np.arange(nz + 1)
    groups = []
    for g in p.dir_u:
        nodes = (g.nodes[None, :] + P * layers[:, None]).reshape(-1)
        groups.append(DirichletU(nodes, np.tile(g.comps, nz + 1), np.tile(g.values, nz + 1)))
    faces = np.concatenate([np.arange(P), np.arange(P) + nz * P])
    groups.append(DirichletU(faces, np.full(faces.size, 2, np.int8), np.zeros(faces.size)))
    dnodes = (p.dir_d_nodes[None, :] + P * layers[:, None]).reshape(-1)
    return Problem3D(name=p.name + "_slab", nx=p.nx, ny=p.ny, nz=nz, lx=p.lx, ly=p.ly, lz=lz,
                     material=p.material, dir_u=groups, dir_d_nodes=dnodes,
                     dir_d_values=np.tile(p.dir_d_values, nz + 1), loads=p.loads.copy(),
                     load_group=p.load_group, load_comp=p.load_comp, tol_stag=p.tol_stag,
                     tol_pcg=p.tol_pcg, tol_newton=p.tol_newton, max_stag=p.max_stag,
                     max_newton=p.max_newton, psi_crit=p.psi_crit, d_gate=p.d_gate,
                     trial_floor=p.trial_floor)


def uniaxial_bar3d(n=3, l=0.03, du=5e-3, steps=6, E=2.1e5, nu=0.3, Gc=2.7) -> Problem3D:
    """Unit cube on rollers (u_x = 0 on x = 0, u_y = 0 on y = 0, u_z = 0 on
    z = 0), top face y = 1 pulled by u_y = lambda: uniaxial stress."""
    nx = ny = nz = n
    P = (nx + 1) * (ny + 1)
    k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    ids = (i + j * (nx + 1) + k * P).reshape(-1)
    i, j, k = i.reshape(-1), j.reshape(-1), k.reshape(-1)
    nodes = np.concatenate([ids[i == 0], ids[j == 0], ids[k == 0]])
    comps = np.concatenate([np.zeros((i == 0).sum()), np.ones((j == 0).sum()),
                            np.full((k == 0).sum(), 2)]).astype(np.int8)
    fixed = DirichletU(nodes, comps, np.zeros(nodes.size))
    top = ids[j == ny]
    pull = DirichletU(top, np.ones(top.size, np.int8), np.ones(top.size))
    return Problem3D(name="bar3d", nx=nx, ny=ny, nz=nz, lx=1.0, ly=1.0, lz=1.0,
                     material=Material(E=E, nu=nu, Gc=Gc, l=l, eta=1e-6),
                     dir_u=[fixed, pull], dir_d_nodes=np.zeros(0, np.int64),
                     dir_d_values=np.zeros(0), loads=du * np.arange(1, steps + 1, dtype=np.float64))


def tilted_notched_box3d(n=4, nz=2, du=3e-3, steps=2, l=0.25) -> Problem3D:
    """A notched box (n x n x nz elements, 1 x 1 x 0.5): bottom face fixed,
    top face pulled by u_y = lambda (0.5 + z/lz), i.e. more at the back than
    at the front, a half-width notch (d = 1) on the mid plane y = 0.5, the
    remaining faces free.  Its fields vary through the thickness, unlike
    those of the extruded slab (uniform in z) and the cube (homogeneous)."""
    lx = ly = 1.0
    lz = 0.5
    P = (n + 1) * (n + 1)
    k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(n + 1), np.arange(n + 1), indexing="ij")
    ids = (i + j * (n + 1) + k * P).reshape(-1)
    i, j, k = i.reshape(-1), j.reshape(-1), k.reshape(-1)
    bot = ids[j == 0]
    fixed = DirichletU(np.repeat(bot, 3), np.tile(np.array([0, 1, 2], np.int8), bot.size),
                       np.zeros(3 * bot.size))
    top = j == n
    pull = DirichletU(ids[top], np.ones(top.sum(), np.int8), 0.5 + k[top] / nz)
    notch = ids[(j == n // 2) & (i <= n // 2)]
    return Problem3D(name="tilted_box", nx=n, ny=n, nz=nz, lx=lx, ly=ly, lz=lz,
                     material=Material(l=l), dir_u=[fixed, pull],
                     dir_d_nodes=notch.astype(np.int64), dir_d_values=np.ones(notch.size),
                     loads=du * np.arange(1, steps + 1, dtype=np.float64))


# --------------------------------------------------------------------------
# Named configurations
# --------------------------------------------------------------------------

def config_tension64(steps=20) -> Problem:
    """64^2 notched tension panel, 20 steps of 3e-4 mm, l = 0.03 mm."""
    return tension_panel(n=64, l=0.03, du=3e-4, steps=steps, name="tension64")


def config_tension512(steps=100) -> Problem:
    """512^2 notched tension panel, 100 steps of 6e-5 mm, l = 0.004 mm."""
    return tension_panel(n=512, l=0.004, du=6e-5, steps=steps, name="tension512")


def config_shear1024(steps=150) -> Problem:
    return shear_panel(n=1024, l=0.004, du=1e-4, steps=steps, name="shear1024")


def config_lshape2048(steps=200) -> Problem:
    return lshape_panel(n=2048, steps=steps, name="lshape2048")


def batch_instances(count=64, seed=2209, steps=50, du=1.6e-4,
                    sizes=(128, 192, 256, 384, 512)):
    """Seeded sweep of notched tension instances.

    Per instance, drawn in this order: mesh size n, Gc (log-uniform in [1,5]),
    the l multiplier (2 or 4 times h) and the notch length a ~ U(0.3, 0.6).
    The notch end is snapped down to the node row grid.
    """
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        n = int(rng.choice(np.asarray(sizes)))
        Gc = float(np.exp(rng.uniform(np.log(1.0), np.log(5.0))))
        mult = int(rng.choice(np.asarray([2, 4])))
        a = float(rng.uniform(0.3, 0.6))
        h = 1.0 / n
        out.append(tension_panel(n=n, l=mult * h, du=du, steps=steps, notch=a,
                                 Gc=Gc, name=f"batch{k}_n{n}"))
    return out


def batch_instance_table(**kw):
    """The drawn parameters of batch_instances(**kw), one dict per instance
    (mesh size, Gc, l, notch length as snapped to the node grid, steps)."""
    rows = []
    for p in batch_instances(**kw):
        notch_x = float(p.dir_d_nodes.max() % (p.nx + 1)) / p.nx
        rows.append({"name": p.name, "n": p.nx, "Gc": p.material.Gc, "l": p.material.l,
                     "notch_end": notch_x, "steps": int(p.loads.size),
                     "du": float(p.loads[0])})
    return rows


def write_batch_instance_table(path, **kw):
    """Record the sweep's instances as JSON (workloads/sweep64_instances.json
    is this function's output for the defaults)."""
    with open(path, "w") as f:
        json.dump({"generator": "numpy.random.default_rng(2209), drawn per instance in the "
                                "order n, Gc, l multiplier, notch length",
                   "instances": batch_instance_table(**kw)}, f, indent=1)
        f.write("\n")


def problem_to_json(p: Problem) -> str:
    d = {
        "name": p.name, "nx": p.nx, "ny": p.ny, "lx": p.lx, "ly": p.ly,
        "material": dataclasses.asdict(p.material),
        "n_dir_u_groups": len(p.dir_u),
        "n_dir_d": int(p.dir_d_nodes.size),
        "loads": [float(x) for x in p.loads[:3]] + ["..."],
        "n_steps": int(p.loads.size),
    }
    return json.dumps(d)
