"""Seeded synthetic inputs for the tDPD + RBC workloads.

This module only draws and lays out inputs: particle positions, velocities,
concentrations, type/frozen flags, a triangulated red-cell surface and where
the cells sit in the box.  It contains none of the method's arithmetic (no
forces, fluxes, weights, rest lengths, areas or volumes), so the GPU library
and the CPU oracle can both be fed from it without sharing any of the
computation they are compared on.

Workload shapes follow the paper's benchmark systems (pure tDPD fluid and RBC
suspensions with 500 membrane particles per cell, Section 5, Table 1): a plain
fluid (c1), one cell in a periodic box (c2), a wall-bounded suspension (c3),
batched ensembles of uneven boxes (ensemble) and a large suspension (c5).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Particle type indices used by every configuration below.
T_SOLVENT = 0
T_MEMBRANE = 1
T_WALL = 2
FLAG_FROZEN = 1 << 8  # flags word: bits 0-7 type index, bit 8 frozen


@dataclass
class MeshParams:
    """Membrane parameters (Section 2.2): WLC persistence length p, rest
    extension ratio x0 = l0/l_m, POW exponent m, bending constant k_b with
    spontaneous angle theta0 (NaN means the mean dihedral of the reference
    shape), global/local area and volume constants, membrane viscosities."""
    p: float = 0.02
    x0: float = 1.0 / 2.2
    m_pow: float = 2.0
    kb: float = 60.0
    theta0: float = float("nan")
    kg: float = 5000.0
    kl: float = 100.0
    kv: float = 5000.0
    gamma_t: float = 3.0
    gamma_c: float = 1.0


@dataclass
class Config:
    name: str
    box: tuple
    rc: float = 1.0
    rcc: float = 1.58
    dt: float = 0.01
    kT: float = 1.0
    rho: float = 3.0
    m_s: float = 0.0
    s_exp: float = 0.25
    sc_exp: float = 2.0
    n_types: int = 3
    n_species: int = 1
    alpha: np.ndarray = None   # [T,T]
    gamma: np.ndarray = None   # [T,T]
    sigma: np.ndarray = None   # [T,T]
    kappa: np.ndarray = None   # [S,T,T]
    body_force: tuple = (0.0, 0.0, 0.0)
    wall_axis: int = -1        # 0-2: planar walls across that axis; 3: cylinder along x
    wall_w: float = 0.0
    wall_radius: float = 0.0   # cylinder radius (wall_axis 3)
    source: np.ndarray = None  # [S,T] zero-order source rate of Q^S (None: 0)
    decay: np.ndarray = None   # [S,T] first-order decay rate of Q^S (None: 0)
    shear_rate: float = 0.0
    seed: int = 1
    box_id: int = 0
    steps: int = 100
    # state, in gid order
    pos: np.ndarray = None     # float32 [N,3]
    vel: np.ndarray = None     # float32 [N,3]
    conc: np.ndarray = None    # float32 [N,S]
    flags: np.ndarray = None   # uint32 [N]
    # membranes: one reference mesh, instances bound to contiguous gid ranges
    mesh_xyz: np.ndarray = None   # float64 [nv,3] reference (rest) shape
    mesh_tri: np.ndarray = None   # int32 [ntri,3], outward counter-clockwise
    mesh_params: MeshParams = field(default_factory=MeshParams)
    rbc_first_gid: list = field(default_factory=list)

    @property
    def n(self):
        return 0 if self.pos is None else int(self.pos.shape[0])


# ---------------------------------------------------------------- state draws
def uniform_positions(n, box, rng):
    box = np.asarray(box, dtype=np.float64)
    x = rng.random((n, 3)) * box
    x = x.astype(np.float32)
    # float32 rounding may land a coordinate on L; fold it back to 0
    for a in range(3):
        L = np.float32(box[a])
        x[x[:, a] >= L, a] = 0.0
    return x


def maxwell_velocities(n, kT, rng, mobile=None):
    v = rng.normal(0.0, math.sqrt(kT), size=(n, 3))
    if mobile is None:
        mobile = np.ones(n, dtype=bool)
    if mobile.any():
        v[mobile] -= v[mobile].mean(axis=0)
    v[~mobile] = 0.0
    return v.astype(np.float32)


def uniform_concentrations(n, n_species, rng):
    return rng.random((n, n_species)).astype(np.float32)


# ---------------------------------------------------------------- RBC surface
def fibonacci_sphere(nv):
    """nv nearly uniform points on the unit sphere (golden-angle spiral)."""
    i = np.arange(nv, dtype=np.float64) + 0.5
    z = 1.0 - 2.0 * i / nv
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def sphere_mesh(nv):
    """Triangulated unit sphere with nv vertices: convex hull of the spiral
    points, every triangle ordered counter-clockwise seen from outside."""
    from scipy.spatial import ConvexHull
    xyz = fibonacci_sphere(nv)
    hull = ConvexHull(xyz)
    tri = hull.simplices.astype(np.int64).copy()
    a, b, c = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    outward = np.einsum("ij,ij->i", np.cross(b - a, c - a), a + b + c) > 0
    tri[~outward] = tri[~outward][:, [0, 2, 1]]
    return xyz, tri.astype(np.int32)


def biconcave_map(xyz_unit, d0=7.8, a=(0.0518, 2.0026, -4.491)):
    """Map unit-sphere points onto the Evans-Fung biconcave disc of diameter
    d0: the azimuth is kept, the in-plane radius scales to d0/2 and the height
    follows the disc's thickness profile."""
    x, y, z = xyz_unit[:, 0], xyz_unit[:, 1], xyz_unit[:, 2]
    u = (x * x + y * y) / 4.0             # rho^2 / d0^2 after scaling
    h = d0 * z * (a[0] + a[1] * u + a[2] * u * u)
    return np.stack([0.5 * d0 * x, 0.5 * d0 * y, h], axis=1)


def rbc_template(nv=500, d0=7.8):
    xyz, tri = sphere_mesh(nv)
    return biconcave_map(xyz, d0), tri


def tetra_mesh():
    xyz = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=np.float64)
    tri = np.array([[0, 1, 2], [0, 3, 1], [0, 2, 3], [1, 3, 2]], dtype=np.int32)
    return xyz, _orient_outward(xyz, tri)


def icosahedron_mesh(edge=1.0):
    """Regular icosahedron with the given edge length (12 vertices, 20 faces)."""
    g = (1.0 + math.sqrt(5.0)) / 2.0
    v = []
    for s1 in (-1, 1):
        for s2 in (-1, 1):
            v += [(0, s1, s2 * g), (s1, s2 * g, 0), (s2 * g, 0, s1)]
    xyz = np.array(v, dtype=np.float64) * (edge / 2.0)
    from scipy.spatial import ConvexHull
    tri = ConvexHull(xyz).simplices.astype(np.int32)
    return xyz, _orient_outward(xyz, tri)


def _orient_outward(xyz, tri):
    tri = tri.astype(np.int64).copy()
    a, b, c = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    cen = xyz.mean(axis=0)
    out = np.einsum("ij,ij->i", np.cross(b - a, c - a), (a + b + c) / 3.0 - cen) > 0
    tri[~out] = tri[~out][:, [0, 2, 1]]
    return tri.astype(np.int32)


def random_rotation(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def place_cells(template, n_cells, box, rng, lo=None, hi=None, min_sep=0.9,
                max_tries=200000):
    """Random sequential placement of rigidly rotated copies of the template
    inside [lo, hi) (per axis), rejecting any copy whose vertices come closer
    than min_sep to an already placed vertex (distances periodic in every
    axis).  Returns a list of [nv,3] float64 arrays.

    A try is checked only against the placed copies whose centre lies within
    two template radii plus min_sep (in any periodic image), each through its
    own k-d tree, so the cost of a try does not grow with the number placed."""
    from scipy.spatial import cKDTree
    box = np.asarray(box, dtype=np.float64)
    lo = np.zeros(3) if lo is None else np.asarray(lo, dtype=np.float64)
    hi = box.copy() if hi is None else np.asarray(hi, dtype=np.float64)
    periodic = (lo <= 0) & (hi >= box)
    radius = float(np.linalg.norm(template - template.mean(axis=0), axis=1).max())
    reach = 2.0 * radius + min_sep
    # periodic images of a neighbour's centre that can come within reach
    shifts = np.stack(np.meshgrid(*[np.arange(-2, 3)] * 3, indexing="ij"), -1).reshape(-1, 3)
    shifts = shifts * box
    placed, centres, trees = [], np.zeros((0, 3)), []
    tries = 0
    while len(placed) < n_cells:
        tries += 1
        if tries > max_tries:
            raise RuntimeError(f"could only place {len(placed)} of {n_cells} cells")
        rot = random_rotation(rng)
        pts = template @ rot.T
        ext_lo, ext_hi = pts.min(axis=0), pts.max(axis=0)
        c = np.empty(3)
        ok = True
        for a in range(3):
            if periodic[a]:
                c[a] = rng.random() * box[a]
            else:
                a0, a1 = lo[a] - ext_lo[a] + 0.5, hi[a] - ext_hi[a] - 0.5
                if a1 <= a0:
                    ok = False
                    break
                c[a] = a0 + rng.random() * (a1 - a0)
        if not ok:
            continue
        pts = pts + c
        cen = pts.mean(axis=0)
        clash = False
        if len(centres):
            d = cen - centres
            d -= box * np.round(d / box)
            for j in np.nonzero(np.linalg.norm(d, axis=1) < reach + 1e-9)[0]:
                # every image of the try that can reach copy j (a coarse
                # subset of its vertices first rejects most clashes cheaply)
                base = cen - (centres[j] + d[j])  # the try moved next to copy j
                near = shifts[np.linalg.norm(d[j] + shifts, axis=1) < reach + 1e-9]
                for sub in (pts[::16], pts):
                    q = (sub - base)[None, :, :] + near[:, None, :]
                    dist, _ = trees[j].query(q.reshape(-1, 3), k=1, distance_upper_bound=min_sep)
                    if np.isfinite(dist).any():
                        clash = True
                        break
                if clash:
                    break
        if clash:
            continue
        placed.append(pts)
        centres = np.concatenate([centres, cen[None]])
        trees.append(cKDTree(pts))
    return placed


# ---------------------------------------------------------------- parameters
def pair_tables(n_types, n_species, a=25.0, g=4.5, s=3.0, kappa=1.0,
                permeability=None, wall_type=None):
    alpha = np.full((n_types, n_types), a)
    gamma = np.full((n_types, n_types), g)
    sigma = np.full((n_types, n_types), s)
    kap = np.full((n_species, n_types, n_types), kappa, dtype=np.float64)
    if permeability is not None:
        for sp, pf in enumerate(permeability):
            kap[sp, T_SOLVENT, T_MEMBRANE] = kappa * pf
            kap[sp, T_MEMBRANE, T_SOLVENT] = kappa * pf
    if wall_type is not None:
        kap[:, wall_type, :] = 0.0
        kap[:, :, wall_type] = 0.0
    return alpha, gamma, sigma, kap


# ---------------------------------------------------------------- configs
def make_fluid(box=(10.0, 10.0, 10.0), rho=4.0, seed=1, n_species=1, n=None,
               steps=100, **kw):
    """Plain periodic tDPD fluid: uniform positions, Maxwellian velocities,
    concentrations uniform in [0,1] (configuration C1 at the defaults)."""
    rng = np.random.default_rng(seed)
    vol = float(np.prod(box))
    n = int(round(rho * vol)) if n is None else n
    alpha, gamma, sigma, kap = pair_tables(3, n_species)
    cfg = Config(name="fluid", box=tuple(float(b) for b in box), rho=rho,
                 n_species=n_species, alpha=alpha, gamma=gamma, sigma=sigma,
                 kappa=kap, seed=seed, steps=steps)
    for k, v in kw.items():
        setattr(cfg, k, v)
    cfg.pos = uniform_positions(n, box, rng)
    cfg.vel = maxwell_velocities(n, cfg.kT, rng)
    cfg.conc = uniform_concentrations(n, n_species, rng)
    cfg.flags = np.full(n, T_SOLVENT, dtype=np.uint32)
    return cfg


def c1(seed=1):
    return make_fluid(box=(10.0, 10.0, 10.0), rho=4.0, seed=seed, n_species=1,
                      steps=100)


def _suspension(name, box, rho, n_cells, seed, n_species=2, walls=False,
                body_force=(0.0, 0.0, 0.0), permeability=(1.0, 0.1), steps=100,
                nv=500, d0=7.8, wall_w=2.0):
    rng = np.random.default_rng(seed)
    box = tuple(float(b) for b in box)
    n_solv = int(round(rho * float(np.prod(box))))
    xs = uniform_positions(n_solv, box, rng)
    flags_s = np.full(n_solv, T_SOLVENT, dtype=np.uint32)
    lo = hi = None
    if walls:
        yy = xs[:, 1]
        frozen = (yy < wall_w) | (yy > box[1] - wall_w)
        flags_s[frozen] = T_WALL | FLAG_FROZEN
        lo = (0.0, wall_w, 0.0)
        hi = (box[0], box[1] - wall_w, box[2])
    tmpl_xyz, tmpl_tri = rbc_template(nv, d0)
    cells = place_cells(tmpl_xyz, n_cells, box, rng, lo=lo, hi=hi) if n_cells else []
    nv = tmpl_xyz.shape[0]
    n = n_solv + nv * len(cells)
    pos = np.empty((n, 3), dtype=np.float32)
    pos[:n_solv] = xs
    flags = np.empty(n, dtype=np.uint32)
    flags[:n_solv] = flags_s
    first = []
    for ci, pts in enumerate(cells):
        g0 = n_solv + ci * nv
        first.append(g0)
        w = np.mod(pts, np.asarray(box)).astype(np.float32)
        for a in range(3):
            w[w[:, a] >= np.float32(box[a]), a] = 0.0
        pos[g0:g0 + nv] = w
        flags[g0:g0 + nv] = T_MEMBRANE
    mobile = (flags & FLAG_FROZEN) == 0
    vel = maxwell_velocities(n, 1.0, rng, mobile)
    conc = np.zeros((n, n_species), dtype=np.float32)
    conc[:, 0] = rng.random(n).astype(np.float32)
    if n_species > 1:
        conc[n_solv:, 1] = 1.0   # the cells carry species 1 (source)
    alpha, gamma, sigma, kap = pair_tables(
        3, n_species, permeability=permeability[:n_species],
        wall_type=T_WALL if walls else None)
    cfg = Config(name=name, box=box, rho=rho, n_species=n_species, alpha=alpha,
                 gamma=gamma, sigma=sigma, kappa=kap, body_force=body_force,
                 wall_axis=1 if walls else -1, wall_w=wall_w if walls else 0.0,
                 seed=seed, steps=steps)
    cfg.pos, cfg.vel, cfg.conc, cfg.flags = pos, vel, conc, flags
    cfg.mesh_xyz, cfg.mesh_tri = tmpl_xyz, tmpl_tri
    cfg.rbc_first_gid = first
    return cfg


def c2(seed=2):
    """Single 500-vertex RBC in a periodic 20^3 box of density-3 solvent,
    two species (species 1 released by the membrane)."""
    return _suspension("single_rbc", (20.0, 20.0, 20.0), 3.0, 1, seed, steps=1000)


def c2_species(n_species=10, seed=2):
    """The single-RBC box with n_species species (the paper's many-species
    regime); the membrane permeability alternates 1.0, 0.1 over species."""
    perm = tuple(1.0 if sp % 2 == 0 else 0.1 for sp in range(n_species))
    return _suspension("single_rbc_species", (20.0, 20.0, 20.0), 3.0, 1, seed,
                       n_species=n_species, permeability=perm, steps=1000)


def c3(seed=3, scale=1.0, n_cells=None, steps=10000):
    """RBC suspension in a wall-bounded channel: 64x32x32 at density 3,
    100 cells, frozen walls in y, body force 0.02 along x.  `scale` shrinks
    the x extent (and the cell count) for small test versions."""
    lx = 64.0 * scale
    nc = int(round(100 * scale)) if n_cells is None else n_cells
    return _suspension("poiseuille_suspension", (lx, 32.0, 32.0), 3.0, nc, seed,
                       walls=True, body_force=(0.02, 0.0, 0.0), steps=steps)


def small_suspension(seed=7, box=(12.0, 12.0, 12.0), n_cells=1, nv=500,
                     walls=False, rho=3.0, d0=7.8):
    return _suspension("small_suspension", box, rho, n_cells, seed, walls=walls,
                       body_force=(0.02, 0.0, 0.0) if walls else (0.0, 0.0, 0.0),
                       nv=nv, d0=d0)


def c5(seed=5, n_cells=1000):
    """Large suspension used for the surrogate-membrane configuration:
    96x96x72 at density 3 plus 1000 cells."""
    return _suspension("large_suspension", (96.0, 96.0, 72.0), 3.0, n_cells, seed,
                       steps=100)


def cylinder(radius=20.0, length=80.0, rho=4.0, seed=9, wall=2.0, c0=0.0, c_wall=1.0,
             kappa=5.0, moving=True, steps=10000):
    """Diffusion in a long tube with a Dirichlet wall (the paper's transport
    validation, Section 4: radius 20, length 80, density 4, alpha 18.75,
    gamma 4.5, r_c = r_cc = 1.58, s = 0.41, flux exponent 2, kappa 5).
    Uniform positions at density rho fill a box of length `length` and width
    2 (radius + wall); particles farther than `radius` from the x-parallel
    axis through the box centre are frozen wall particles that hold the wall
    concentration c_wall (and exchange flux with the fluid: kappa to the wall
    as to the fluid), the fluid starts at c0.  moving=False gives the fluid
    zero velocities (run with the force terms off, the particles then stay
    in place: the pure-diffusion case)."""
    rng = np.random.default_rng(seed)
    w = 2.0 * (radius + wall)
    box = (float(length), w, w)
    n = int(round(rho * float(np.prod(box))))
    pos = uniform_positions(n, box, rng)
    dy = pos[:, 1].astype(np.float64) - 0.5 * w
    dz = pos[:, 2].astype(np.float64) - 0.5 * w
    outside = dy * dy + dz * dz > radius * radius
    flags = np.full(n, T_SOLVENT, dtype=np.uint32)
    flags[outside] = T_WALL | FLAG_FROZEN
    mobile = ~outside
    vel = maxwell_velocities(n, 1.0, rng, mobile)
    if not moving:
        vel[:] = 0.0
    conc = np.full((n, 1), c0, dtype=np.float32)
    conc[outside, 0] = c_wall
    alpha, gamma, sigma, kap = pair_tables(3, 1, a=18.75, g=4.5, s=3.0, kappa=kappa)
    cfg = Config(name="cylinder", box=box, rc=1.58, rcc=1.58, rho=rho, s_exp=0.41,
                 sc_exp=2.0, n_species=1, alpha=alpha, gamma=gamma, sigma=sigma,
                 kappa=kap, wall_axis=3, wall_radius=float(radius), seed=seed,
                 steps=steps)
    cfg.pos, cfg.vel, cfg.conc, cfg.flags = pos, vel, conc, flags
    return cfg


def ensemble_sizes(n_boxes=256, lo=2000, hi=60000, seed=4):
    rng = np.random.default_rng(seed)
    return np.round(np.exp(rng.uniform(math.log(lo), math.log(hi), n_boxes))).astype(int)


def ensemble(n_boxes=256, seed=4, lo=2000, hi=60000, rho=3.0, max_cells=4, shear_max=0.5):
    """Batched-ensemble workload: n_boxes independent periodic cubic boxes of
    log-uniform particle count in [lo, hi] at density rho, each with its own
    seed (1000 + b), box id b, shear rate U[0, shear_max] and U{0..max_cells}
    cells (none where the box is narrower than 12, at most 20 % of the box
    volume).  One species.  Returns a list of Config, one per box."""
    rng = np.random.default_rng(seed)
    sizes = np.round(np.exp(rng.uniform(math.log(lo), math.log(hi), n_boxes))).astype(int)
    shears = rng.uniform(0.0, shear_max, n_boxes)
    ncells = rng.integers(0, max_cells + 1, n_boxes)
    boxes = []
    for b in range(n_boxes):
        L = float((sizes[b] / rho) ** (1.0 / 3.0))
        nc = int(ncells[b]) if L >= 12.0 else 0
        nc = min(nc, int(0.2 * L ** 3 / 95.0))
        cfg = _suspension(f"ensemble_{b}", (L, L, L), rho, nc, 1000 + b, n_species=1,
                          permeability=(1.0,))
        cfg.seed = 1000 + b
        cfg.box_id = b
        cfg.shear_rate = float(shears[b])
        boxes.append(cfg)
    return boxes


# ---------------------------------------------------------------- surrogate
SURR_SHAPES = [(128, 20), (128, 128), (128, 128), (3, 128)]


def mlp_init_params(seed=0):
    """Seeded initial parameters of the membrane-surrogate network, flat in
    the layer order [W1, b1, W2, b2, W3, b3, W4, b4]: normal weights with
    standard deviation sqrt(2 / fan_in), zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for no, ni in SURR_SHAPES:
        parts.append(rng.normal(0.0, math.sqrt(2.0 / ni), no * ni))
        parts.append(np.zeros(no))
    return np.concatenate(parts).astype(np.float32)
