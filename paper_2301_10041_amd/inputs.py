"""Seeded synthetic inputs shared by the FP64 oracle and the HIP path.

This module holds none of the method's arithmetic.  It produces, on the host, the
arrays that both sides receive unchanged (so both see bit-identical inputs):

* the reference mesh of the immersed solid (a concentric-ring disk or its affine
  image, an ellipse), with counter-clockwise P1 triangles;
* seeded right-hand sides and velocities drawn uniformly in [-1, 1];
* prescribed solid positions X^n for the time loop (a rigid rotation);
* the arrival trace of the request loop (exponential inter-arrival times).

The paper does not specify its meshes (Sec. 6 uses a quarter annulus and a bar on
Q1 meshes that are not published); the workloads below are synthetic stand-ins with
the paper's size ratios (solid elements about as large as fluid cells).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def ring_disk(m: int, center=(0.5, 0.5), radius: float = 0.2, semi_axes=None):
    """P1 mesh of a disk made of ``m`` concentric rings of nodes.

    Node 0 is the centre; ring k (1..m) holds 6k nodes at radius k/m (unit disk)
    at angles 2*pi*i/(6k).  Between rings k-1 and k there are 6(2k-1) triangles,
    so the mesh has 6m^2 triangles and 3m^2+3m+1 nodes.  The unit disk is scaled
    by ``radius`` (or by ``semi_axes=(a, b)`` for an ellipse) and shifted to
    ``center``.  Returns ``(xy, tri)``: float64 [Ns, 2] and int32 [Nt, 3] (CCW).
    """
    if m < 1:
        raise ValueError("m must be >= 1")
    start = [0]
    for k in range(1, m + 1):
        start.append(1 + 3 * (k - 1) * k)          # first node of ring k
    nn = 3 * m * m + 3 * m + 1
    ux = np.zeros(nn)
    uy = np.zeros(nn)
    for k in range(1, m + 1):
        i = np.arange(6 * k)
        ang = 2.0 * np.pi * i / (6 * k)
        ux[start[k]:start[k] + 6 * k] = (k / m) * np.cos(ang)
        uy[start[k]:start[k] + 6 * k] = (k / m) * np.sin(ang)
    tris = []
    for k in range(1, m + 1):
        nout = 6 * k
        nin = 6 * (k - 1)

        def outer(t):
            return start[k] + (t % nout)

        def inner(t):
            return 0 if k == 1 else start[k - 1] + (t % nin)

        for s in range(6):
            for t in range(k):                      # outer edge + inner vertex
                tris.append((outer(s * k + t), outer(s * k + t + 1), inner(s * (k - 1) + t)))
            for t in range(k - 1):                  # inner edge + outer vertex
                tris.append((inner(s * (k - 1) + t), outer(s * k + t + 1), inner(s * (k - 1) + t + 1)))
    tri = np.asarray(tris, dtype=np.int32)
    if semi_axes is None:
        a = b = float(radius)
    else:
        a, b = float(semi_axes[0]), float(semi_axes[1])
    xy = np.empty((nn, 2))
    xy[:, 0] = center[0] + a * ux
    xy[:, 1] = center[1] + b * uy
    return xy, tri


def bar_mesh(nx: int, ny: int, x0=0.0, x1=0.4, y0=0.45, y1=0.55):
    """P1 mesh of the rectangle [x0, x1] x [y0, y1] (the bar of the nonlinear test, Sec. 6.2):
    nx x ny cells, each split along (i, j) -> (i + 1, j + 1) into two counter-clockwise
    triangles.  Node (i, j) has index j (nx + 1) + i.  Returns ``(xy, tri)``."""
    xs = x0 + (x1 - x0) * np.arange(nx + 1) / nx
    ys = y0 + (y1 - y0) * np.arange(ny + 1) / ny
    X, Y = np.meshgrid(xs, ys, indexing="xy")
    xy = np.stack([X.ravel(), Y.ravel()], axis=1)
    tris = []
    for j in range(ny):
        for i in range(nx):
            a, b = j * (nx + 1) + i, j * (nx + 1) + i + 1
            c, d = (j + 1) * (nx + 1) + i + 1, (j + 1) * (nx + 1) + i
            tris.append((a, b, c))
            tris.append((a, c, d))
    return xy, np.asarray(tris, dtype=np.int32)


def quad_bar(nx: int, ny: int, x0=0.3, x1=0.7, y0=0.45, y1=0.55):
    """Q1 mesh of the rectangle [x0, x1] x [y0, y1]: nx x ny rectangular cells, node (i, j) at
    index j (nx + 1) + i, quadrilateral (i, j), (i + 1, j), (i + 1, j + 1), (i, j + 1)
    (counter-clockwise) with index j nx + i.  Returns ``(xy, quad)``: float64 [Ns, 2] and
    int32 [Nq, 4]."""
    xs = x0 + (x1 - x0) * np.arange(nx + 1) / nx
    ys = y0 + (y1 - y0) * np.arange(ny + 1) / ny
    X, Y = np.meshgrid(xs, ys, indexing="xy")
    xy = np.stack([X.ravel(), Y.ravel()], axis=1)
    quads = []
    for j in range(ny):
        for i in range(nx):
            a = j * (nx + 1) + i
            quads.append((a, a + 1, a + nx + 2, a + nx + 1))
    return xy, np.asarray(quads, dtype=np.int32)


def bent(xy: np.ndarray, amp: float, length: float = 0.4, x0: float = 0.0) -> np.ndarray:
    """A released position of the bar: every point moved down by amp ((s_x - x0) / length)^2 (a
    bending that leaves the left end in place)."""
    out = xy.copy()
    out[:, 1] = xy[:, 1] - amp * ((xy[:, 0] - x0) / length) ** 2
    return out


def uniform(n: int, seed: int) -> np.ndarray:
    """``n`` float64 values uniform in [-1, 1) from ``numpy.random.default_rng(seed)``."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, n)


def rotation(xy: np.ndarray, center, angle: float) -> np.ndarray:
    """Prescribed rigid rotation of the reference positions about ``center``."""
    c, s = math.cos(angle), math.sin(angle)
    dx = xy[:, 0] - center[0]
    dy = xy[:, 1] - center[1]
    out = np.empty_like(xy)
    out[:, 0] = center[0] + c * dx - s * dy
    out[:, 1] = center[1] + s * dx + c * dy
    return out


@dataclass
class Solid:
    """One immersed body: a ring disk (or ellipse) mesh."""
    m: int
    center: tuple
    radius: float = 0.2
    semi_axes: tuple | None = None

    def mesh(self):
        return ring_disk(self.m, self.center, self.radius, self.semi_axes)


@dataclass
class Bar(Solid):
    """The bar [x0, x0 + 0.4] x [0.45, 0.55] of the nonlinear test with nx x ny cells (x0 = 0 is
    the paper's position against the wall)."""
    nx: int = 16
    ny: int = 4
    x0: float = 0.0

    def mesh(self):
        return bar_mesh(self.nx, self.ny, self.x0, self.x0 + 0.4)


@dataclass
class Workload:
    """A synthetic FSI workload: fluid grid, immersed solids and parameters."""
    name: str
    n: int
    solids: list = field(default_factory=list)
    nu: float = 1.0
    rho: float = 1.0
    kappa: float = 10.0
    dt: float = 0.01
    seed: int = 0

    def solid_mesh(self):
        """Concatenate the bodies into one reference mesh (node ids offset)."""
        xs, ts, off = [], [], 0
        for s in self.solids:
            xy, tri = s.mesh()
            xs.append(xy)
            ts.append(tri + off)
            off += xy.shape[0]
        return np.concatenate(xs, axis=0), np.concatenate(ts, axis=0).astype(np.int32)

    def sizes(self):
        n = self.n
        xy, tri = self.solid_mesh()
        n2 = (2 * n + 1) ** 2
        np_ = (n + 1) ** 2
        ns = xy.shape[0]
        return dict(N2=n2, Np=np_, Ns=ns, Nt=tri.shape[0], N=2 * n2 + np_ + 4 * ns)


# The five workloads (sizes and seeds) of the evaluation; see the design doc for the recipe.
WORKLOADS = {
    # 32^2 fluid, disk R=0.2 at the centre with 216 triangles, block-diagonal, seed 0
    "disk32": Workload("disk32", 32, [Solid(6, (0.5, 0.5), 0.2)], dt=0.01, seed=0),
    # 256^2 fluid, ellipse 0.25 x 0.15 at (0.45, 0.55), 12,150 triangles, seed 1
    "ellipse256": Workload("ellipse256", 256, [Solid(45, (0.45, 0.55), semi_axes=(0.25, 0.15))],
                           dt=0.01, seed=1),
    # 512^2 fluid, disk R=0.2, 40,344 triangles, rotation 0.1 rad/s, dt=1e-3, 100 steps
    "rotdisk512": Workload("rotdisk512", 512, [Solid(82, (0.5, 0.5), 0.2)], dt=1e-3, seed=2),
    # the 1024^2 two-disk geometry on a 128^2 grid (ring count scaled with the grid: m = 14,
    # 1,176 triangles per disk), seed 3: the mid-size parity case and the CPU baseline sample
    "twodisk128": Workload("twodisk128", 128,
                           [Solid(14, (0.3, 0.5), 0.1), Solid(14, (0.7, 0.5), 0.1)],
                           dt=0.01, seed=3),
    # the 512^2 rotating-disk time loop on a 256^2 grid (ring count scaled with the grid: m = 41,
    # 10,086 triangles), dt = 1e-3: the size at which the oracle's exact block factorisations of
    # the time loop still fit the host (its first-step iteration count)
    "rotdisk256": Workload("rotdisk256", 256, [Solid(41, (0.5, 0.5), 0.2)], dt=1e-3, seed=2),
    # 1024^2 fluid, two disks R=0.1 at (0.3,0.5), (0.7,0.5), 75,264 triangles each, seed 3
    "twodisk1024": Workload("twodisk1024", 1024,
                            [Solid(112, (0.3, 0.5), 0.1), Solid(112, (0.7, 0.5), 0.1)],
                            dt=0.01, seed=3),
}


# the nonlinear test's bar (Sec. 6.2: 0.4 x 0.1, nu = 0.2, rho = 1, dt = 0.002) on a 256^2 grid
# with solid cells of the fluid cell size (102 x 26 cells, 5,304 triangles), moved 0.05 off the
# wall x = 0 (the clipping needs X^n(B) inside the square and nothing holds the left end on the
# wall), released from a bent position with u^0 = 0
WORKLOADS["bar256"] = Workload("bar256", 256, [Bar(m=0, center=(0.25, 0.5), nx=102, ny=26, x0=0.05)], nu=0.2,
                               rho=1.0, kappa=1.333, dt=0.002, seed=5)


@dataclass
class QWorkload:
    """A workload of the paper's own element pair (Sec. 4: Q2 velocity, discontinuous P1
    pressure, Q1 solid): an n x n fluid grid and one bar [x0, x1] x [y0, y1] with nx x ny
    quadrilaterals."""
    name: str
    n: int
    nx: int
    ny: int
    x0: float = 0.3
    x1: float = 0.7
    y0: float = 0.45
    y1: float = 0.55
    nu: float = 1.0
    rho: float = 1.0
    kappa: float = 10.0
    dt: float = 0.01
    seed: int = 0

    def solid_mesh(self):
        return quad_bar(self.nx, self.ny, self.x0, self.x1, self.y0, self.y1)

    @property
    def center(self):
        return (0.5 * (self.x0 + self.x1), 0.5 * (self.y0 + self.y1))

    def sizes(self):
        n = self.n
        ns = (self.nx + 1) * (self.ny + 1)
        n2 = (2 * n + 1) ** 2
        np_ = 3 * n * n
        return dict(N2=n2, Np=np_, Ns=ns, Nt=self.nx * self.ny, N=2 * n2 + np_ + 4 * ns)


# the paper's element pair on the bar of the nonlinear test: 0.4 x 0.1 with quadrilaterals of
# the fluid cell size, nu = 0.2, dt = 0.002 (Sec. 6.2), the linear law kappa = 10; qbar32 the
# parity case, qbar256 the measured one (102 x 26 quadrilaterals)
QWORKLOADS = {
    "qbar32": QWorkload("qbar32", 32, 13, 3, nu=0.2, dt=0.002, seed=7),
    "qbar256": QWorkload("qbar256", 256, 102, 26, nu=0.2, dt=0.002, seed=7),
}


def small_workload(n: int, m: int, center=(0.5, 0.5), radius=0.2, semi_axes=None,
                   dt=0.01, seed=0, nu=1.0, rho=1.0, kappa=10.0) -> Workload:
    """A workload of arbitrary (small) size for tests."""
    return Workload(f"n{n}m{m}", n, [Solid(m, center, radius, semi_axes)], nu=nu, rho=rho,
                    kappa=kappa, dt=dt, seed=seed)


def request_trace(count: int = 512, rate: float = 200.0, seed: int = 4):
    """Open-loop request trace of the request loop.

    Exponential inter-arrival times with mean 1/rate seconds; per request a grid
    size n in {32, 64, 128, 256}, a disk or an ellipse (probability 1/2 each) with
    centre uniform in [0.3, 0.7]^2, radius uniform in [0.05, 0.2] (ellipse minor
    semi-axis scaled by U[0.6, 1]) and ring count m uniform in {6..45}
    (216 to 12,150 triangles).  Request i draws its right-hand side from seed 1000+i.
    """
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, count))
    t -= t[0]
    out = []
    for i in range(count):
        n = int(rng.choice([32, 64, 128, 256]))
        ellipse = bool(rng.random() < 0.5)
        cx, cy = rng.uniform(0.3, 0.7, 2)
        r = float(rng.uniform(0.05, 0.2))
        m = int(rng.integers(6, 46))
        ratio = float(rng.uniform(0.6, 1.0))
        axes = (r, r * ratio) if ellipse else None
        wl = Workload(f"req{i}", n, [Solid(m, (float(cx), float(cy)), r, axes)], dt=0.01,
                      seed=1000 + i)
        out.append((float(t[i]), wl))
    return out
