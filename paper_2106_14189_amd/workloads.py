"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds mesh geometry, random draws and load descriptions only --
none of the DJ-TLED arithmetic -- so that the GPU path and the CPU oracle can
be fed the same inputs.  The paper's own meshes (a cube with circular
cut-outs, Sec. 5.1; a brain mesh, Sec. 6) are not available; these stand in:

* ``cube_mesh``: a jittered structured grid of voxels, each split into six
  linear tetrahedra (Kuhn/Freudenthal split, conforming) or kept as one
  8-node hexahedron.  Node orders follow the conventions of the library:
  T4 with positive det under h = (1 - xi - eta - zeta, xi, eta, zeta); H8 in
  (---, +--, ++-, -+-, --+, +-+, +++, -++) order.
* ``ellipsoid_mesh``: voxelised ellipsoid, Kuhn-split, interior jitter.
* load descriptions: bottom face fixed, top face z-displacement ramped.

Seeds follow ``210614189 + 1000 * config + instance``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 210614189

T4, H8 = 4, 8
NH, TI, OT, MR = 0, 1, 2, 3
RAMP_NONE, RAMP_LINEAR, RAMP_SMOOTH = 0, 1, 2


def seed_for(config: int, instance: int = 0) -> int:
    return SEED_BASE + 1000 * config + instance


@dataclass
class Mesh:
    X: np.ndarray            # (N, 3) float64 reference coordinates
    conn: np.ndarray         # (E, ne) int32
    bottom: np.ndarray       # node ids on the z = min face
    top: np.ndarray          # node ids on the z = max face
    height: float = 0.0

    @property
    def ne(self) -> int:
        return int(self.conn.shape[1])

    @property
    def n_nodes(self) -> int:
        return int(self.X.shape[0])

    @property
    def n_elems(self) -> int:
        return int(self.conn.shape[0])


@dataclass
class Material:
    model: int
    E: np.ndarray                       # (E,) Young's modulus [Pa]
    nu: np.ndarray                      # (E,) Poisson's ratio
    rho: float = 1000.0
    eta_ratio: np.ndarray | None = None  # (E,) fibre stiffness ratio eta_a / mu (TI, OT)
    fibre: np.ndarray | None = None      # (E, 3) unit fibre directions a (TI, OT)
    hg_kappa: float = 0.1
    eta_b_ratio: np.ndarray | None = None  # (E,) second fibre ratio eta_b / mu (OT)
    fibre_b: np.ndarray | None = None      # (E, 3) unit fibre directions b, orthogonal to a (OT)
    c01: np.ndarray | None = None          # (E,) Mooney-Rivlin C01 [Pa] (MR; C10 = mu / 2)


@dataclass
class Loads:
    bc_node: np.ndarray                 # (nb,) int32
    bc_mask: np.ndarray                 # (nb,) int32, bit k = component k constrained
    bc_target: np.ndarray               # (nb, 3) float64 target displacement at ramp end
    ramp: int = RAMP_SMOOTH
    t_ramp: float = 0.0
    R: np.ndarray | None = None         # (N, 3) external nodal forces or None


@dataclass
class Workload:
    name: str
    mesh: Mesh
    material: Material
    loads: Loads
    dt_factor: float = 0.9
    alpha: float = 0.0
    n_steps: int = 0
    fp64: bool = False
    seed: int = 0
    extra: dict = field(default_factory=dict)


# Kuhn split: the six tetrahedra of a voxel follow the monotone lattice paths
# from corner (0,0,0) to (1,1,1).  Odd permutations get their last two
# vertices swapped so every tetrahedron is positively oriented.
_PERMS = [((0, 1, 2), +1), ((0, 2, 1), -1), ((1, 0, 2), -1),
          ((1, 2, 0), +1), ((2, 0, 1), +1), ((2, 1, 0), -1)]
_H8_CORNERS = [(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)]


def _kuhn_tets():
    tets = []
    for perm, sign in _PERMS:
        c = [0, 0, 0]
        verts = [tuple(c)]
        for ax in perm:
            c[ax] += 1
            verts.append(tuple(c))
        if sign < 0:
            verts[2], verts[3] = verts[3], verts[2]
        tets.append(verts)
    return tets


def _grid_conn(nx, ny, nz, elem, voxel_mask=None):
    def nid(i, j, k):
        return i + (nx + 1) * (j + (ny + 1) * k)

    i, j, k = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    i = i.transpose(2, 1, 0).ravel()
    j = j.transpose(2, 1, 0).ravel()
    k = k.transpose(2, 1, 0).ravel()
    if voxel_mask is not None:
        keep = voxel_mask[i, j, k]
        i, j, k = i[keep], j[keep], k[keep]
    if elem == H8:
        cols = [nid(i + a, j + b, k + c) for (a, b, c) in _H8_CORNERS]
        return np.stack(cols, axis=1).astype(np.int32)
    per = []
    for verts in _kuhn_tets():
        per.append(np.stack([nid(i + a, j + b, k + c) for (a, b, c) in verts], axis=1))
    # voxel-major: the 6 tets of one voxel are consecutive
    return np.stack(per, axis=1).reshape(-1, 4).astype(np.int32)


def cube_mesh(n: int, h: float, elem: int = T4, jitter: float = 0.05, seed: int = 0,
              permute: bool = False) -> Mesh:
    """n^3 voxels of side h.  Interior nodes are jittered uniformly by
    +-jitter*h per coordinate; boundary nodes move only tangentially, so the
    faces stay planar and the total volume stays (n h)^3."""
    rng = np.random.default_rng(seed)
    g = np.arange(n + 1)
    kk, jj, ii = np.meshgrid(g, g, g, indexing="ij")
    idx = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1)      # node id = i + (n+1)(j + (n+1)k)
    X = idx.astype(np.float64) * h
    if jitter > 0:
        d = rng.uniform(-jitter * h, jitter * h, size=X.shape)
        on_bnd = (idx == 0) | (idx == n)
        d[on_bnd] = 0.0
        X = X + d
    conn = _grid_conn(n, n, n, elem)
    bottom = np.nonzero(idx[:, 2] == 0)[0]
    top = np.nonzero(idx[:, 2] == n)[0]
    mesh = Mesh(X=X, conn=conn, bottom=bottom.astype(np.int32), top=top.astype(np.int32), height=n * h)
    if permute:
        mesh = permute_mesh(mesh, rng)
    return mesh


def permute_mesh(mesh: Mesh, rng) -> Mesh:
    """Random relabelling of nodes and elements (mimics unstructured ordering)."""
    N, E = mesh.n_nodes, mesh.n_elems
    pn = rng.permutation(N)            # new id -> old id
    inv = np.empty(N, np.int64)
    inv[pn] = np.arange(N)             # old id -> new id
    pe = rng.permutation(E)
    X = mesh.X[pn]
    conn = inv[mesh.conn[pe]].astype(np.int32)
    return Mesh(X=X, conn=conn, bottom=np.sort(inv[mesh.bottom]).astype(np.int32),
                top=np.sort(inv[mesh.top]).astype(np.int32), height=mesh.height)


def signed_volume6(X, conn):
    """6 x the signed volume of each tetrahedron (mesh validity check only)."""
    a, b, c, d = (X[conn[:, i]] for i in range(4))
    return np.einsum("ij,ij->i", b - a, np.cross(c - a, d - a))


def ellipsoid_mesh(semi=(0.05, 0.04, 0.03), target_elems=1_200_000, jitter=0.15, seed=0,
                   permute=True) -> Mesh:
    """Voxelised ellipsoid: voxels whose centre lies inside are kept and
    Kuhn-split; interior nodes are jittered by +-jitter*h (re-drawn where a
    tetrahedron would lose positive orientation)."""
    rng = np.random.default_rng(seed)
    a, b, c = semi
    vol = 4.0 / 3.0 * np.pi * a * b * c
    h = (vol / (target_elems / 6.0)) ** (1.0 / 3.0)
    n = [int(np.ceil(2 * s / h)) + 2 for s in semi]
    lo = np.array([-s for s in semi]) - h
    ci = (np.arange(n[0]) + 0.5) * h + lo[0]
    cj = (np.arange(n[1]) + 0.5) * h + lo[1]
    ck = (np.arange(n[2]) + 0.5) * h + lo[2]
    I, J, K = np.meshgrid(ci, cj, ck, indexing="ij")
    inside = (I / a) ** 2 + (J / b) ** 2 + (K / c) ** 2 <= 1.0
    conn_full = _grid_conn(n[0], n[1], n[2], T4, inside)
    used = np.unique(conn_full)
    remap = -np.ones((n[0] + 1) * (n[1] + 1) * (n[2] + 1), np.int64)
    remap[used] = np.arange(len(used))
    conn = remap[conn_full].astype(np.int32)
    gi = used % (n[0] + 1)
    gj = (used // (n[0] + 1)) % (n[1] + 1)
    gk = used // ((n[0] + 1) * (n[1] + 1))
    X = np.stack([gi, gj, gk], axis=1).astype(np.float64) * h + lo
    # boundary nodes: those belonging to a voxel face that is not shared
    counts = np.zeros(len(used), np.int64)
    np.add.at(counts, conn.ravel(), 1)
    interior = counts == 24  # a Kuhn-interior node touches 24 tetrahedra
    if jitter > 0:
        for _ in range(8):
            d = rng.uniform(-jitter * h, jitter * h, size=X.shape)
            d[~interior] = 0.0
            Xn = X + d
            bad = signed_volume6(Xn, conn) <= 0.05 * h ** 3
            if not bad.any():
                X = Xn
                break
            # keep the draw except at nodes of bad elements
            badn = np.unique(conn[bad])
            d[badn] = 0.0
            Xn = X + d
            if (signed_volume6(Xn, conn) > 0).all():
                X = Xn
                break
    zmin = X[:, 2].min()
    bottom = np.nonzero((X[:, 2] < -0.8 * c) & ~interior)[0]
    top = np.nonzero((X[:, 2] > 0.8 * c) & ~interior)[0]
    mesh = Mesh(X=X, conn=conn, bottom=bottom.astype(np.int32), top=top.astype(np.int32),
                height=float(X[:, 2].max() - zmin))
    mesh.surface = np.nonzero(~interior)[0].astype(np.int32)
    mesh.h = h
    if permute:
        pn = rng.permutation(mesh.n_nodes)
        inv = np.empty(mesh.n_nodes, np.int64)
        inv[pn] = np.arange(mesh.n_nodes)
        pe = rng.permutation(mesh.n_elems)
        m2 = Mesh(X=mesh.X[pn], conn=inv[mesh.conn[pe]].astype(np.int32),
                  bottom=np.sort(inv[mesh.bottom]).astype(np.int32),
                  top=np.sort(inv[mesh.top]).astype(np.int32), height=mesh.height)
        m2.surface = np.sort(inv[mesh.surface]).astype(np.int32)
        m2.h = h
        mesh = m2
    return mesh


def compression_loads(mesh: Mesh, strain: float = -0.2, ramp=RAMP_SMOOTH, t_ramp=0.0) -> Loads:
    """Bottom face fixed in all components; top face z-displacement ramped to
    strain * height (x and y free)."""
    nb = len(mesh.bottom)
    nt = len(mesh.top)
    bc_node = np.concatenate([mesh.bottom, mesh.top]).astype(np.int32)
    bc_mask = np.concatenate([np.full(nb, 7), np.full(nt, 4)]).astype(np.int32)
    tgt = np.zeros((nb + nt, 3))
    tgt[nb:, 2] = strain * mesh.height
    return Loads(bc_node=bc_node, bc_mask=bc_mask, bc_target=tgt, ramp=ramp, t_ramp=t_ramp)


def uniform_material(n_elems, E, nu, rho=1000.0, model=NH, rng=None, eta_ratio_range=(2.0, 10.0),
                     c01_ratio_range=(0.2, 1.0)):
    """Material of one model.  TI/OT: fibre a uniform on the sphere and
    eta_a / mu ~ U(eta_ratio_range); OT adds b uniform on the circle orthogonal
    to a and eta_b / mu from the same range; MR: C01 / C10 ~ U(c01_ratio_range)
    with C10 = mu / 2."""
    E = np.broadcast_to(np.asarray(E, np.float64), (n_elems,)).copy()
    nu = np.broadcast_to(np.asarray(nu, np.float64), (n_elems,)).copy()
    mat = Material(model=model, E=E, nu=nu, rho=rho)
    rng = rng or np.random.default_rng(0)
    if model in (TI, OT):
        v = rng.normal(size=(n_elems, 3))
        mat.fibre = v / np.linalg.norm(v, axis=1, keepdims=True)
        mat.eta_ratio = rng.uniform(*eta_ratio_range, size=n_elems)
    if model == OT:
        w = rng.normal(size=(n_elems, 3))
        w -= np.sum(w * mat.fibre, axis=1, keepdims=True) * mat.fibre
        mat.fibre_b = w / np.linalg.norm(w, axis=1, keepdims=True)
        mat.eta_b_ratio = rng.uniform(*eta_ratio_range, size=n_elems)
    if model == MR:
        mu = E / (2.0 * (1.0 + nu))
        mat.c01 = rng.uniform(*c01_ratio_range, size=n_elems) * mu / 2.0
    return mat


# ---------------------------------------------------------------------------
# The benchmark configurations
# ---------------------------------------------------------------------------

def config0(seed_offset: int = 0) -> Workload:
    """10^3 voxels of 0.01 m, 6 tets each (6000 T4 / 1331 nodes), NH E=3000 Pa,
    nu=0.45, rho=1000; bottom fixed, top z ramped smoothly to -20 % of the
    height over the run; dt = 0.9 x critical; 2000 steps; FP64."""
    seed = seed_for(0) + seed_offset
    mesh = cube_mesh(10, 0.01, T4, jitter=0.05, seed=seed)
    mat = uniform_material(mesh.n_elems, 3000.0, 0.45, 1000.0)
    loads = compression_loads(mesh, -0.2, RAMP_SMOOTH)
    # damping: alpha = 2 omega_hat, omega_hat = pi c_s / (2 L) with c_s = sqrt(mu / rho)
    return Workload("cube10_t4_nh_fp64", mesh, mat, loads, 0.9, alpha=32.0, n_steps=2000, fp64=True, seed=seed)


def config1(elem: int = T4, n: int = 64, n_steps: int = 1000, seed_offset: int = 0) -> Workload:
    """64^3 voxels over a 0.1 m cube as 1,572,864 T4 or 262,144 H8 (274,625
    nodes); E ~ U[2, 6] kPa per element, nu = 0.45, rho = 1000; jitter +-5 %;
    elements and nodes randomly permuted; config-0 compression load; FP32."""
    seed = seed_for(1) + seed_offset + (0 if elem == T4 else 500)
    rng = np.random.default_rng(seed + 7)
    mesh = cube_mesh(n, 0.1 / n, elem, jitter=0.05, seed=seed, permute=True)
    E = rng.uniform(2000.0, 6000.0, size=mesh.n_elems)
    mat = uniform_material(mesh.n_elems, E, 0.45, 1000.0)
    loads = compression_loads(mesh, -0.2, RAMP_SMOOTH)
    name = f"cube{n}_{'t4' if elem == T4 else 'h8'}_nh_fp32"
    return Workload(name, mesh, mat, loads, 0.9, alpha=37.0, n_steps=n_steps, fp64=False, seed=seed)


def patch_loads(mesh: Mesh, rng, frac: float = 0.05, amp: float = 0.003, n_rbf: int = 4, width: float = 1.0,
                ramp=RAMP_SMOOTH, t_ramp=0.0, fix_bottom: bool = True) -> Loads:
    """Bottom cap fixed; about `frac` of the surface nodes, in one seeded patch
    around a random upper-surface node, prescribed with a smooth field: a sum of
    `n_rbf` Gaussian radial basis functions (width `width` x R) with random
    vector weights, times the window (1 - (r / R)^2)^2 that vanishes at the
    patch rim (r: distance from the patch centre, R: patch radius), scaled to
    a maximum magnitude of `amp`.  The window alone stretches the surface by
    up to 1.54 amp / R; amp = 3 mm on the R ~ 18 mm patch keeps the prescribed
    stretch near 25 %."""
    surf = mesh.surface
    Xs = mesh.X[surf]
    upper = surf[Xs[:, 2] > 0.0]
    centre = mesh.X[rng.choice(upper)]
    d = np.linalg.norm(mesh.X[surf] - centre, axis=1)
    k = max(4, int(round(frac * len(surf))))
    patch = surf[np.argsort(d)[:k]]
    P = mesh.X[patch]
    radius = np.linalg.norm(P - centre, axis=1).max() + 1e-12
    centres = P[rng.choice(len(patch), n_rbf, replace=False)]
    weights = rng.normal(size=(n_rbf, 3))
    field = np.zeros((len(patch), 3))
    for c, w in zip(centres, weights):
        field += np.exp(-np.sum((P - c) ** 2, axis=1) / (width * radius) ** 2)[:, None] * w[None, :]
    r = np.linalg.norm(P - centre, axis=1) / radius
    field *= ((1.0 - r * r) ** 2)[:, None]
    field *= amp / np.linalg.norm(field, axis=1).max()
    fixed = np.setdiff1d(mesh.bottom, patch) if fix_bottom else np.zeros(0, np.int32)
    bc_node = np.concatenate([fixed, patch]).astype(np.int32)
    bc_mask = np.full(len(bc_node), 7, np.int32)
    tgt = np.concatenate([np.zeros((len(fixed), 3)), field])
    return Loads(bc_node=bc_node, bc_mask=bc_mask, bc_target=tgt, ramp=ramp, t_ramp=t_ramp)


def config2(target_elems: int = 1_200_000, seed_offset: int = 0) -> Workload:
    """Transversely isotropic neo-Hookean ellipsoid (semi-axes 0.05, 0.04,
    0.03 m) voxelised into ~1.2M Kuhn tetrahedra, interior nodes jittered
    +-15 %, nodes and elements permuted; E = 3 kPa, nu = 0.45, rho = 1000;
    per-element unit fibre uniform on the sphere, eta_a / mu ~ U[2, 10];
    bottom cap (z < -0.8 c) fixed; ~5 % of the surface nodes prescribed with a
    smooth windowed random field of maximum 3 mm, ramped smoothly over 0.4 s;
    dynamic relaxation to 1e-6."""
    seed = seed_for(2) + seed_offset
    rng = np.random.default_rng(seed)
    mesh = ellipsoid_mesh(target_elems=target_elems, jitter=0.15, seed=seed, permute=True)
    mat = uniform_material(mesh.n_elems, 3000.0, 0.45, 1000.0, model=TI, rng=rng)
    loads = patch_loads(mesh, rng)
    wl = Workload(f"ellipsoid{mesh.n_elems // 1000}k_t4_ti_fp32_relax", mesh, mat, loads, 0.9, alpha=60.0,
                  n_steps=200000, fp64=False, seed=seed)
    wl.extra.update(t_ramp=0.4, tol=1e-6, check_every=100)
    return wl


def box_mesh(nx: int, ny: int, nz: int, h: float, elem: int = T4, jitter: float = 0.05, seed: int = 0) -> Mesh:
    """nx x ny x nz voxels of side h, jittered like cube_mesh (boundary nodes
    move only tangentially, so the faces stay planar)."""
    rng = np.random.default_rng(seed)
    kk, jj, ii = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    idx = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1)  # node id = i + (nx+1)(j + (ny+1)k)
    X = idx.astype(np.float64) * h
    if jitter > 0:
        d = rng.uniform(-jitter * h, jitter * h, size=X.shape)
        d[(idx == 0) | (idx == np.array([nx, ny, nz]))] = 0.0
        X = X + d
    conn = _grid_conn(nx, ny, nz, elem)
    bottom = np.nonzero(idx[:, 2] == 0)[0].astype(np.int32)
    top = np.nonzero(idx[:, 2] == nz)[0].astype(np.int32)
    return Mesh(X=X, conn=conn, bottom=bottom, top=top, height=nz * h)


def box_instance(E_target: int, elem: int, model: int, rng, size: float = 0.1, jitter: float = 0.05,
                 permute: bool = True):
    """A jittered, permuted box grid with about E_target elements (6 Kuhn
    tetrahedra or one hexahedron per voxel), n x n x nz voxels of side
    size / n, with E ~ U[2, 6] kPa per element, nu = 0.45, and for TI a unit
    fibre uniform on the sphere and eta_a / mu ~ U[2, 10]."""
    vox = E_target / (6.0 if elem == T4 else 1.0)
    n = max(2, int(round(vox ** (1.0 / 3.0))))
    nz = max(2, int(round(vox / (n * n))))
    m = box_mesh(n, n, nz, size / n, elem, jitter=jitter, seed=int(rng.integers(2 ** 31)))
    if permute:
        m = permute_mesh(m, rng)
    mat = uniform_material(m.n_elems, rng.uniform(2000.0, 6000.0, m.n_elems), 0.45, 1000.0, model=model, rng=rng)
    return m, mat


def config3(n_inst: int = 256, n_steps: int = 500, seed_offset: int = 0, e_min: float = 5e3, e_max: float = 2e5):
    """Batch of independent box instances: element counts log-uniform in
    [5k, 200k], element kind (T4 / H8) and model (NH / TI) each a fair coin;
    bottom face fixed, top face moved by a displacement of magnitude U[5 %,
    20 %] of the height in a seeded direction (downward z component), smooth
    ramp over the run's steps.  Returns a list of (Mesh, Material, Loads,
    alpha) with t_ramp given in steps (negative)."""
    out = []
    for k in range(n_inst):
        rng = np.random.default_rng(seed_for(3, k) + seed_offset)
        Ek = int(round(np.exp(rng.uniform(np.log(e_min), np.log(e_max)))))
        elem = T4 if rng.random() < 0.5 else H8
        model = NH if rng.random() < 0.5 else TI
        mesh, mat = box_instance(Ek, elem, model, rng)
        d = rng.normal(size=3)
        d[2] = -abs(d[2]) - 0.5
        d /= np.linalg.norm(d)
        amp = rng.uniform(0.05, 0.20) * mesh.height
        nb, nt = len(mesh.bottom), len(mesh.top)
        loads = Loads(bc_node=np.concatenate([mesh.bottom, mesh.top]).astype(np.int32),
                      bc_mask=np.full(nb + nt, 7, np.int32),
                      bc_target=np.concatenate([np.zeros((nb, 3)), np.tile(amp * d, (nt, 1))]),
                      ramp=RAMP_SMOOTH, t_ramp=-float(n_steps))
        out.append((mesh, mat, loads, 37.0))
    return out
