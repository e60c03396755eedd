"""Terrain-following tetrahedral meshes of a shallow basin (data generation only).

The domain is the shallow region of Sec. 2: a horizontal surface Gamma_s (here
the rectangle [0,Lx] x [0,Ly]) over a depth h(x1,x2) > 0, i.e.
{(x1,x2) in Gamma_s, -h(x1,x2) < x3 < 0}.  Its boundary below the surface,
Gamma_b, is the bottom plus the four lateral walls; Gamma_b splits into the
Dirichlet part Gamma_0 and the artificial part Gamma_1 (Sec. 2 and the boundary
conditions of the prediction step in Sec. 3).

Mesh recipe (the paper meshes with hexahedra, Sec. 5; the main path uses
linear tetrahedra cut from the same cells, HexMesh below keeps the bricks):
  * nodes (i,j,k), 0<=i<=Nx, 0<=j<=Ny, 0<=k<=Nz, uniform sigma layers:
      x = i*Lx/Nx,  y = j*Ly/Ny,  z = -h(x,y)*(1 - k/Nz)
    so k = 0 is the bottom and k = Nz the surface z = 0;
  * node numbering is vertical-first: id = (i*(Ny+1) + j)*(Nz+1) + k, so each
    water column is a contiguous run of Nz+1 ids;
  * each hexahedral cell is cut into the 6 Kuhn (Freudenthal) tetrahedra, one
    per monotone lattice path from corner (0,0,0) to corner (1,1,1); the cut is
    the same in every cell, so the mesh is conforming.  Tetrahedra are oriented
    positively (det[v1-v0, v2-v0, v3-v0] > 0) by swapping the last two vertices
    of the paths of odd permutations;
  * the surface triangles are the top faces of the top cells, each surface
    square split along its (i,j)-(i+1,j+1) diagonal (the faces the Kuhn cut
    leaves on the plane k = Nz).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# Dirichlet bits carried per node.  Bit c marks the nodes where velocity
# component c+1 is prescribed to zero:
#   u1: Gamma_0                 (no slip)
#   u2: Gamma_0 + Gamma_1       (no normal flow through the south/north limits)
#   u3: Gamma_0 + Gamma_s       (u3 = 0 on the surface)
BC_U1 = 1
BC_U2 = 2
BC_U3 = 4

# The six Kuhn paths: permutations of the axes (0 = i, 1 = j, 2 = k) with
# their parity.
_KUHN_PATHS = (
    ((0, 1, 2), +1), ((1, 2, 0), +1), ((2, 0, 1), +1),
    ((0, 2, 1), -1), ((1, 0, 2), -1), ((2, 1, 0), -1),
)

WALLS = ("bottom", "west", "east", "south", "north")


def node_index(i, j, k, Ny: int, Nz: int):
    """Vertical-first node id of lattice point (i, j, k)."""
    return (np.asarray(i, dtype=np.int64) * (Ny + 1) + j) * (Nz + 1) + k


@dataclass
class BasinMesh:
    """A structured terrain-following tetrahedral mesh and its boundary data.

    xyz       (n, 3) float64, metres (or unit-less for the unit box)
    tets      (n_tets, 4) int32, 0-based node ids, positively oriented
    bc        (n,) uint8, Dirichlet bits BC_U1 | BC_U2 | BC_U3
    surf_tris (n_surf, 3) int32, the surface triangles on z = 0
    depth     ((Nx+1)*(Ny+1),) float64, h at the water columns (i-major)
    """
    Nx: int
    Ny: int
    Nz: int
    Lx: float
    Ly: float
    xyz: np.ndarray
    tets: np.ndarray
    bc: np.ndarray
    surf_tris: np.ndarray
    depth: np.ndarray
    gamma0: tuple = field(default=("bottom", "west", "east"))
    gamma1: tuple = field(default=("south", "north"))

    @property
    def n(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_tets(self) -> int:
        return int(self.tets.shape[0])

    def free_mask(self, bit: int) -> np.ndarray:
        """Boolean (n,) array, True where the node is not Dirichlet for `bit`."""
        return (self.bc & bit) == 0


def _lattice(Nx: int, Ny: int, Nz: int):
    i, j, k = np.meshgrid(np.arange(Nx + 1), np.arange(Ny + 1),
                          np.arange(Nz + 1), indexing="ij")
    return i.ravel(), j.ravel(), k.ravel()


def kuhn_tets(Nx: int, Ny: int, Nz: int) -> np.ndarray:
    """Connectivity of the 6*Nx*Ny*Nz Kuhn tetrahedra, cell-major order."""
    ci, cj, ck = np.meshgrid(np.arange(Nx), np.arange(Ny), np.arange(Nz),
                             indexing="ij")
    ci, cj, ck = ci.ravel(), cj.ravel(), ck.ravel()
    out = np.empty((ci.size, 6, 4), dtype=np.int64)
    for t, (perm, parity) in enumerate(_KUHN_PATHS):
        corner = np.zeros(3, dtype=np.int64)
        verts = [corner.copy()]
        for axis in perm:
            corner[axis] += 1
            verts.append(corner.copy())
        if parity < 0:
            verts[2], verts[3] = verts[3], verts[2]
        for v, off in enumerate(verts):
            out[:, t, v] = node_index(ci + off[0], cj + off[1], ck + off[2], Ny, Nz)
    return out.reshape(-1, 4).astype(np.int32)


def surface_triangles(Nx: int, Ny: int, Nz: int) -> np.ndarray:
    ci, cj = np.meshgrid(np.arange(Nx), np.arange(Ny), indexing="ij")
    ci, cj = ci.ravel(), cj.ravel()
    a = node_index(ci, cj, Nz, Ny, Nz)
    b = node_index(ci + 1, cj, Nz, Ny, Nz)
    c = node_index(ci + 1, cj + 1, Nz, Ny, Nz)
    d = node_index(ci, cj + 1, Nz, Ny, Nz)
    tris = np.empty((ci.size, 2, 3), dtype=np.int64)
    tris[:, 0] = np.stack([a, b, c], axis=1)
    tris[:, 1] = np.stack([a, c, d], axis=1)
    return tris.reshape(-1, 3).astype(np.int32)


def dirichlet_bits(Nx: int, Ny: int, Nz: int, gamma0=("bottom", "west", "east"),
                   gamma1=("south", "north")) -> np.ndarray:
    """Per-node Dirichlet bits for a given split of Gamma_b into Gamma_0/Gamma_1.

    A node belongs to a face if it lies on it; corner and edge nodes belong to
    every face they touch.
    """
    for name in tuple(gamma0) + tuple(gamma1):
        if name not in WALLS:
            raise ValueError(f"unknown boundary face {name!r}")
    i, j, k = _lattice(Nx, Ny, Nz)
    on = {
        "bottom": k == 0, "west": i == 0, "east": i == Nx,
        "south": j == 0, "north": j == Ny,
    }
    surface = k == Nz
    g0 = np.zeros(i.size, dtype=bool)
    for name in gamma0:
        g0 |= on[name]
    g1 = np.zeros(i.size, dtype=bool)
    for name in gamma1:
        g1 |= on[name]
    bits = np.zeros(i.size, dtype=np.uint8)
    bits[g0] |= BC_U1
    bits[g0 | g1] |= BC_U2
    bits[g0 | surface] |= BC_U3
    return bits


def bathymetry(x, y, L: float, seed: int, n_bumps: int = 32,
               h_min: float = 200.0, h_max: float = 5500.0) -> np.ndarray:
    """Seeded stand-in for the basin depth (the real bathymetry is not available).

    h = 200 m + sum of n_bumps Gaussian bumps, clipped to [h_min, h_max]; the
    bump centres, amplitudes and widths are drawn as arrays in the order
    cx ~ U[0,L], cy ~ U[0,L], a ~ U[500,5300] m, s ~ U[100,600] km.
    """
    rng = np.random.default_rng(seed)
    cx = rng.uniform(0.0, L, n_bumps)
    cy = rng.uniform(0.0, L, n_bumps)
    a = rng.uniform(500.0, 5300.0, n_bumps)
    s = rng.uniform(100e3, 600e3, n_bumps)
    x = np.asarray(x, dtype=np.float64)[..., None]
    y = np.asarray(y, dtype=np.float64)[..., None]
    bumps = a * np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2.0 * s ** 2))
    return np.clip(200.0 + bumps.sum(axis=-1), h_min, h_max)


def _build(Nx, Ny, Nz, Lx, Ly, depth_fn, gamma0, gamma1) -> BasinMesh:
    if min(Nx, Ny, Nz) < 1:
        raise ValueError("need at least one cell in each direction")
    i, j, k = _lattice(Nx, Ny, Nz)
    x = i * (Lx / Nx)
    y = j * (Ly / Ny)
    ci, cj = np.meshgrid(np.arange(Nx + 1), np.arange(Ny + 1), indexing="ij")
    depth = np.asarray(depth_fn(ci.ravel() * (Lx / Nx), cj.ravel() * (Ly / Ny)),
                       dtype=np.float64)
    if np.any(depth <= 0):
        raise ValueError("depth must be positive")
    col = i * (Ny + 1) + j
    z = -depth[col] * (1.0 - k / Nz)
    xyz = np.stack([x, y, z], axis=1).astype(np.float64)
    return BasinMesh(Nx=Nx, Ny=Ny, Nz=Nz, Lx=float(Lx), Ly=float(Ly), xyz=xyz,
                     tets=kuhn_tets(Nx, Ny, Nz),
                     bc=dirichlet_bits(Nx, Ny, Nz, gamma0, gamma1),
                     surf_tris=surface_triangles(Nx, Ny, Nz), depth=depth,
                     gamma0=tuple(gamma0), gamma1=tuple(gamma1))


def box_mesh(Nx: int, Ny: int, Nz: int, Lx: float = 1.0, Ly: float = 1.0,
             H: float = 0.01, gamma0=WALLS, gamma1=()) -> BasinMesh:
    """Flat-bottomed box [0,Lx] x [0,Ly] x [-H, 0] (the small plain-method case).

    By default all of Gamma_b (bottom and four walls) is Dirichlet.
    """
    return _build(Nx, Ny, Nz, Lx, Ly, lambda x, y: np.full_like(x, H, dtype=np.float64),
                  gamma0, gamma1)


def basin_mesh(Nx: int, Ny: int, Nz: int, L: float = 5.0e6, seed: int = 0,
               gamma0=("bottom", "west", "east"),
               gamma1=("south", "north")) -> BasinMesh:
    """Square basin of side L over the seeded Gaussian-bump bathymetry.

    The default boundary split follows the North-Atlantic set-up of Sec. 6:
    continents (no slip) to the west and east, artificial limits (no normal
    flow) at the Equator (south) and 70N (north), no slip at the bottom.
    """
    return _build(Nx, Ny, Nz, L, L, lambda x, y: bathymetry(x, y, L, seed),
                  gamma0, gamma1)


@dataclass
class HexMesh:
    """A structured terrain-following hexahedral mesh of order 1 (Q1) or 2 (Q2).

    The elements are the Nx x Ny x Nz cells of the recipe above (the brick
    elements of Sec. 5).  The nodes are the lattice of the refined grid
    (order*Nx+1) x (order*Ny+1) x (order*Nz+1), numbered vertical-first like
    the tetrahedral meshes, so water columns stay contiguous runs of
    order*Nz+1 ids.  Each cell is the trilinear image of the reference cube
    through its 8 corners; the other Q2 nodes sit at the images of the
    reference nodes (mid-edge, mid-face and centre), so the refined lattice's
    depth is the bilinear interpolant of the corner depths within each cell.

    hexes     (n_hex, (order+1)**3) int32; local node (a, b, c), a along x,
              b along y, c along z (each in 0..order), at column
              a + (order+1)*b + (order+1)**2*c
    bc        Dirichlet bits on the refined lattice (same split as the
              tetrahedral meshes)
    depth     ((order*Nx+1)*(order*Ny+1),) depth at the refined columns
    """
    Nx: int
    Ny: int
    Nz: int
    order: int
    Lx: float
    Ly: float
    xyz: np.ndarray
    hexes: np.ndarray
    bc: np.ndarray
    depth: np.ndarray
    gamma0: tuple = field(default=("bottom", "west", "east"))
    gamma1: tuple = field(default=("south", "north"))

    @property
    def n(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_hex(self) -> int:
        return int(self.hexes.shape[0])

    @property
    def line_len(self) -> int:
        return self.order * self.Nz + 1


def _build_hex(Nx, Ny, Nz, order, Lx, Ly, depth_fn, gamma0, gamma1) -> HexMesh:
    if min(Nx, Ny, Nz) < 1:
        raise ValueError("need at least one cell in each direction")
    if order not in (1, 2):
        raise ValueError("order must be 1 or 2")
    p = order
    Mx, My, Mz = p * Nx, p * Ny, p * Nz
    # corner depths, then their bilinear interpolant on the refined columns
    ci, cj = np.meshgrid(np.arange(Nx + 1), np.arange(Ny + 1), indexing="ij")
    hc = np.asarray(depth_fn(ci.ravel() * (Lx / Nx), cj.ravel() * (Ly / Ny)),
                    dtype=np.float64).reshape(Nx + 1, Ny + 1)
    if np.any(hc <= 0):
        raise ValueError("depth must be positive")
    fi, fj = np.meshgrid(np.arange(Mx + 1), np.arange(My + 1), indexing="ij")
    i0 = np.minimum(fi // p, Nx - 1)
    j0 = np.minimum(fj // p, Ny - 1)
    s = (fi - p * i0) / p
    t = (fj - p * j0) / p
    h = ((1 - s) * (1 - t) * hc[i0, j0] + s * (1 - t) * hc[i0 + 1, j0]
         + (1 - s) * t * hc[i0, j0 + 1] + s * t * hc[i0 + 1, j0 + 1]).ravel()
    i, j, k = _lattice(Mx, My, Mz)
    x = i * (Lx / Mx)
    y = j * (Ly / My)
    z = -h[i * (My + 1) + j] * (1.0 - k / Mz)
    xyz = np.stack([x, y, z], axis=1).astype(np.float64)
    ei, ej, ek = np.meshgrid(np.arange(Nx), np.arange(Ny), np.arange(Nz), indexing="ij")
    ei, ej, ek = ei.ravel(), ej.ravel(), ek.ravel()
    q = p + 1
    hexes = np.empty((ei.size, q ** 3), dtype=np.int64)
    for c in range(q):
        for b in range(q):
            for a in range(q):
                hexes[:, a + q * b + q * q * c] = node_index(p * ei + a, p * ej + b, p * ek + c,
                                                             My, Mz)
    return HexMesh(Nx=Nx, Ny=Ny, Nz=Nz, order=p, Lx=float(Lx), Ly=float(Ly), xyz=xyz,
                   hexes=hexes.astype(np.int32), bc=dirichlet_bits(Mx, My, Mz, gamma0, gamma1),
                   depth=h, gamma0=tuple(gamma0), gamma1=tuple(gamma1))


def box_hex_mesh(Nx: int, Ny: int, Nz: int, order: int, Lx: float = 1.0, Ly: float = 1.0,
                 H: float = 0.01, gamma0=WALLS, gamma1=()) -> HexMesh:
    """Flat-bottomed box [0,Lx] x [0,Ly] x [-H, 0] in brick elements."""
    return _build_hex(Nx, Ny, Nz, order, Lx, Ly,
                      lambda x, y: np.full_like(x, H, dtype=np.float64), gamma0, gamma1)


def basin_hex_mesh(Nx: int, Ny: int, Nz: int, order: int, L: float = 5.0e6, seed: int = 0,
                   gamma0=("bottom", "west", "east"),
                   gamma1=("south", "north")) -> HexMesh:
    """Square basin over the seeded bathymetry, in brick elements of the given order."""
    return _build_hex(Nx, Ny, Nz, order, L, L, lambda x, y: bathymetry(x, y, L, seed),
                      gamma0, gamma1)
