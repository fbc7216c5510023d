"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This module holds input generation only: mesh topology, vertex coordinates,
boundary masks and random vectors/fields.  It contains none of the method's
arithmetic (no quadrature, no basis functions, no geometric factors, no operator),
so that the oracle and the HIP library stay independent of each other.

Mesh recipe (the paper's setting of mapped hexahedra, Section 3, on the unit cube):

* ``ne^3`` hexahedra on [0,1]^3, spacing h = 1/ne.  Interior vertices are moved
  by i.i.d. U(-amp*h, amp*h) per coordinate (amp = 0.1 by default); boundary
  vertices stay put, so the domain is exactly the unit cube.  The element geometry
  is the trilinear map through the 8 vertices.
* Element numbering e = ex + ne*(ey + ne*ez).  Vertex v of an element is the corner
  (i, j, k) in {0,1}^3 with v = i + 2j + 4k (i along x, i.e. along xi_1).
* Global DoF numbering for order p: N1 = ne*p + 1 nodes per direction,
  g = gx + N1*(gy + N1*gz) with gx = ex*p + i etc.  Local element DoF
  l = i + (p+1)*(j + (p+1)*k), i fastest.
* Essential (Dirichlet) DoFs: every DoF on the boundary of the cube.

Seeds (numpy ``default_rng``): mesh 0, x / rhs 1, nu 2, nu* 3, finite-difference
directions 100.., batched nu fields 200...
"""
from __future__ import annotations

import numpy as np

SEED_MESH = 0
SEED_X = 1
SEED_NU = 2
SEED_NU_STAR = 3
SEED_FD_DIR = 100
SEED_NU_BATCH = 200


class BoxMesh:
    """A structured, perturbed ``ne^3`` hex mesh of the unit cube with an order-p DoF map.

    Attributes are plain numpy arrays:
      elem_xyz  [NE, 8, 3] float64   vertex coordinates, vertex v = i + 2j + 4k
      elem_dofs [NE, (p+1)^3] int32  element-to-global DoF map, local l = i + n(j + n k)
      ess       [N] uint8            1 on boundary DoFs
    """

    def __init__(self, ne: int, p: int, amp: float = 0.1, seed: int = SEED_MESH):
        if ne < 1 or p < 1:
            raise ValueError("ne and p must be >= 1")
        self.ne, self.p, self.amp, self.seed = ne, p, amp, seed
        n = p + 1
        self.n = n
        self.nelem = ne ** 3
        n1 = ne * p + 1
        self.n1 = n1
        self.ndof = n1 ** 3

        # vertices of the ne^3 grid, interior ones perturbed
        nv = ne + 1
        h = 1.0 / ne
        g = np.arange(nv) * h
        vx, vy, vz = np.meshgrid(g, g, g, indexing="ij")  # [ix, iy, iz]
        verts = np.stack([vx, vy, vz], axis=-1)  # [nv, nv, nv, 3]
        rng = np.random.default_rng(seed)
        pert = rng.uniform(-amp * h, amp * h, size=verts.shape)
        interior = np.zeros((nv, nv, nv), dtype=bool)
        if nv > 2:
            interior[1:-1, 1:-1, 1:-1] = True
        verts = verts + pert * interior[..., None]

        ex, ey, ez = np.meshgrid(np.arange(ne), np.arange(ne), np.arange(ne), indexing="ij")
        # element id e = ex + ne*(ey + ne*ez): flatten with ex fastest
        ex = ex.transpose(2, 1, 0).reshape(-1)
        ey = ey.transpose(2, 1, 0).reshape(-1)
        ez = ez.transpose(2, 1, 0).reshape(-1)
        xyz = np.empty((self.nelem, 8, 3), dtype=np.float64)
        for v in range(8):
            i, j, k = v & 1, (v >> 1) & 1, (v >> 2) & 1
            xyz[:, v, :] = verts[ex + i, ey + j, ez + k, :]
        self.elem_xyz = xyz

        li = np.arange(n)
        I, J, K = np.meshgrid(li, li, li, indexing="ij")
        # local l = i + n*(j + n*k): order the flattened arrays with i fastest
        I = I.transpose(2, 1, 0).reshape(-1)
        J = J.transpose(2, 1, 0).reshape(-1)
        K = K.transpose(2, 1, 0).reshape(-1)
        gx = ex[:, None] * p + I[None, :]
        gy = ey[:, None] * p + J[None, :]
        gz = ez[:, None] * p + K[None, :]
        self.elem_dofs = (gx + n1 * (gy + n1 * gz)).astype(np.int32)

        gidx = np.arange(n1)
        on_b = (gidx == 0) | (gidx == n1 - 1)
        bx, by, bz = np.meshgrid(on_b, on_b, on_b, indexing="ij")
        ess = (bx | by | bz).transpose(2, 1, 0).reshape(-1)
        self.ess = ess.astype(np.uint8)

    def global_coords_grid(self):
        """Integer grid coordinates (gx, gy, gz) of every global DoF."""
        g = np.arange(self.ndof)
        return g % self.n1, (g // self.n1) % self.n1, g // (self.n1 * self.n1)


class TaylorHoodMesh:
    """Velocity (order p) and pressure (order p - 1) DoF maps on one ``ne^3`` box mesh.

    vel: the order-p BoxMesh (with its boundary mask, the velocity Dirichlet DoFs);
    pres_dofs [NE, p^3] int32 and npres: the order-(p-1) map of the same elements,
    numbered like BoxMesh (no essential pressure DoFs).
    """

    def __init__(self, ne: int, p: int, amp: float = 0.1, seed: int = SEED_MESH):
        if p < 2:
            raise ValueError("the Taylor-Hood pair needs p >= 2")
        self.vel = BoxMesh(ne, p, amp=amp, seed=seed)
        pm = BoxMesh(ne, p - 1, amp=amp, seed=seed)
        if not np.array_equal(pm.elem_xyz, self.vel.elem_xyz):
            raise AssertionError("velocity and pressure meshes differ")
        self.pres_dofs = pm.elem_dofs
        self.npres = pm.ndof
        self.ne, self.p, self.nelem = ne, p, self.vel.nelem


class FanMesh:
    """An unstructured hex mesh: ``nsect`` kite-shaped columns around the z axis, each
    split into ``nlayer`` layers on z in [0, 1], so that the nodes on the axis are
    shared by nsect (inside a layer) or 2 nsect (on a layer interface) elements -- DoF
    multiplicities a structured box mesh does not have.  Section s spans the angles
    [2 pi s / nsect, 2 pi (s + 1) / nsect]; its cross-section has the vertices O (the
    axis), R(theta_s), R(theta_{s+1}) (radius 1) and the outer corner at the middle
    angle (radius ``rc``); vertex v = i + 2j + 4k with i along O -> R(theta_s) and j
    along O -> R(theta_{s+1}), which keeps the map orientation positive for nsect >= 3.

    DoFs are numbered by deduplicating the images of the equispaced lattice
    (i/p, j/p, k/p) under each element's trilinear map (a conforming neighbour sees a
    shared face through a symmetry of the square, so shared nodes coincide).
    Essential DoFs: the nodes on the bottom face z = 0.
    """

    def __init__(self, p: int, nsect: int = 3, nlayer: int = 2, rc: float = 1.0):
        if nsect < 3 or nlayer < 1 or p < 1:
            raise ValueError("need nsect >= 3, nlayer >= 1, p >= 1")
        self.p, self.n = p, p + 1
        n = p + 1
        self.nelem = nsect * nlayer
        xyz = np.empty((self.nelem, 8, 3))
        e = 0
        for layer in range(nlayer):
            for sct in range(nsect):
                t0 = 2 * np.pi * sct / nsect
                t1 = 2 * np.pi * (sct + 1) / nsect
                tm = 0.5 * (t0 + t1)
                quad = {(0, 0): (0.0, 0.0), (1, 0): (np.cos(t0), np.sin(t0)),
                        (0, 1): (np.cos(t1), np.sin(t1)), (1, 1): (rc * np.cos(tm), rc * np.sin(tm))}
                for v in range(8):
                    i, j, k = v & 1, (v >> 1) & 1, (v >> 2) & 1
                    xyz[e, v, :2] = quad[(i, j)]
                    xyz[e, v, 2] = (layer + k) / nlayer
                e += 1
        self.elem_xyz = xyz
        s = np.arange(n) / p
        S1, S2, S3 = np.meshgrid(s, s, s, indexing="ij")  # [i, j, k]
        # lattice point of local l = i + n (j + n k)
        lat = np.stack([S1, S2, S3], -1).transpose(2, 1, 0, 3).reshape(-1, 3)
        keys = {}
        dofs = np.empty((self.nelem, n ** 3), dtype=np.int32)
        coords = []
        for e in range(self.nelem):
            for l in range(n ** 3):
                a, b, c = lat[l]
                w = np.array([(1 - a) * (1 - b) * (1 - c), a * (1 - b) * (1 - c), (1 - a) * b * (1 - c),
                              a * b * (1 - c), (1 - a) * (1 - b) * c, a * (1 - b) * c, (1 - a) * b * c, a * b * c])
                x = w @ xyz[e]
                key = tuple(np.round(x * 1e9).astype(np.int64))
                if key not in keys:
                    keys[key] = len(coords)
                    coords.append(x)
                dofs[e, l] = keys[key]
        self.elem_dofs = dofs
        self.ndof = len(coords)
        self.node_xyz = np.array(coords)
        self.ess = (np.abs(self.node_xyz[:, 2]) < 1e-12).astype(np.uint8)


def uniform(n, seed: int = SEED_X, lo: float = -1.0, hi: float = 1.0, shape=None) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=shape if shape is not None else n)


def normal(n, seed: int = SEED_X) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n)


def rhs_uniform(mesh: BoxMesh, seed: int = SEED_X, nbatch: int = 1) -> np.ndarray:
    """b ~ U(-1,1) on free DoFs, b = 0 on essential DoFs; shape [nbatch, N]."""
    rng = np.random.default_rng(seed)
    b = rng.uniform(-1.0, 1.0, size=(nbatch, mesh.ndof))
    b[:, mesh.ess.astype(bool)] = 0.0
    return b


def nu_uniform(nelem: int, nq1: int, seed: int, lo: float = 0.5, hi: float = 2.0) -> np.ndarray:
    """Per-quadrature-point coefficient field ~ U(lo, hi), layout [nelem, nq1^3]."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(nelem, nq1 ** 3))


def nu_c2(x, y, z):
    """Variable viscosity nu(x) = 1 + 0.5 sin(2 pi x) cos(2 pi y) (works on numpy or torch)."""
    mod = np if isinstance(x, np.ndarray) else __import__("torch")
    return 1.0 + 0.5 * mod.sin(2.0 * np.pi * x) * mod.cos(2.0 * np.pi * y)


def u_manufactured(x, y, z):
    """u = sin(pi x) sin(pi y) sin(pi z); -Laplace(u) = 3 pi^2 u."""
    mod = np if isinstance(x, np.ndarray) else __import__("torch")
    return mod.sin(np.pi * x) * mod.sin(np.pi * y) * mod.sin(np.pi * z)


def f_manufactured(x, y, z):
    return 3.0 * np.pi ** 2 * u_manufactured(x, y, z)


# Named workloads at the sizes the method is exercised on.  Each entry:
# (ne, p, q, description).  q = p + 2 Gauss-Legendre points per direction.
WORKLOADS = {
    "poisson_p2_4e": dict(ne=4, p=2, alpha=0.0, beta=1.0,
                          desc="diffusion apply + Jacobi-PCG Poisson, 4^3 hexes, p=2, nu=1"),
    "helmholtz_p4_32e": dict(ne=32, p=4, alpha=1e3, beta=1.0,
                             desc="Helmholtz 1e3*M + K(nu), nu(x)=1+0.5sin(2pi x)cos(2pi y), 32^3 hexes, p=4"),
    "vector_helmholtz_p7_24e": dict(ne=24, p=7, alpha=1e3, beta=1.0, nbatch=3,
                                    desc="3-component Helmholtz, 24^3 hexes, p=7, FP32 inner + FP64 IR"),
    "adjoint_p5_20e": dict(ne=20, p=5, alpha=1e3, beta=1.0,
                           desc="adjoint dJ/dnu, nu~U(0.5,2) per qpt, 20^3 hexes, p=5"),
    "large_p8_40e": dict(ne=40, p=8, alpha=1e3, beta=1.0,
                         desc="FP32+IR Helmholtz PCG + 4-field batched gradient, 40^3 hexes, p=8"),
}
