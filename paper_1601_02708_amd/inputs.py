"""Seeded synthetic inputs for the hybrid FEM/LBM transport problem.

This module produces *inputs only*: solid geometry, advection velocity,
initial concentration and reaction-rate fields.  It holds none of the
method's arithmetic (no equilibria, no collision, no FEM), so both the
CPU oracle and the GPU path may consume the same arrays.

Geometry conventions (shared by every consumer):

* The whole domain is the square [0, L]^2 in lattice units, L = 2(N-1),
  where N is the number of fine lattice nodes per side.  The fine
  (pore-scale) patch is the central quarter of the unit-square layout,
  i.e. [(N-1)/2, 3(N-1)/2]^2; fine node (i, j) sits at
  (x0 + i, y0 + j) with x0 = y0 = (N-1)/2.
* Fine arrays are row-major [N, N] with j (the y index) as the slow axis.
* Coarse nodal arrays are row-major [(M+1), (M+1)] over the M x M
  bilinear mesh on [0, L]^2 with spacing L/M.

The porous geometry stands in for the paper's calcite workload (circular
solid grains inside a D2Q9 pore domain, Sec. 7.4), whose actual geometry
exists only in the paper's figures.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


# ----------------------------------------------------------------------------
# domain layout
# ----------------------------------------------------------------------------

def domain_side(N: int) -> float:
    """Side of the whole (coarse) domain in lattice units: L = 2(N-1)."""
    return 2.0 * (N - 1)


def patch_origin(N: int) -> float:
    """Domain coordinate of fine node (0, 0) along each axis: (N-1)/2."""
    return 0.5 * (N - 1)


def fine_coords(N: int):
    """Domain coordinates (X, Y) of every fine node, each shaped [N, N]."""
    x0 = patch_origin(N)
    ax = x0 + np.arange(N, dtype=np.float64)
    Y, X = np.meshgrid(ax, ax, indexing="ij")
    return X, Y


def coarse_coords(M: int, L: float):
    """Domain coordinates (X, Y) of every coarse node, each [(M+1), (M+1)]."""
    ax = np.arange(M + 1, dtype=np.float64) * (L / M)
    Y, X = np.meshgrid(ax, ax, indexing="ij")
    return X, Y


# ----------------------------------------------------------------------------
# solid grains: random sequential addition of non-overlapping disks
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class DiskPack:
    solid: np.ndarray        # uint8 [N, N], 1 = solid node
    centers: np.ndarray      # float64 [n, 2] (i, j) lattice coordinates
    radii: np.ndarray        # float64 [n]
    porosity: float          # achieved fluid fraction


def random_disks(N: int, porosity: float, seed: int, r_min: float = 6.0,
                 r_max: float = 20.0, margin: float = 2.0, gap: float = 1.0,
                 max_attempts: int = 5_000_000) -> DiskPack:
    """Random sequential addition of disks until the solid fraction reaches
    1 - porosity.

    Radii are uniform in [r_min, r_max]; centres uniform such that every disk
    stays at least ``margin`` lattice units inside the patch; two disks keep a
    surface gap of at least ``gap``.  A node (i, j) is solid iff its distance
    to some centre is <= r.  The gap guarantees no node belongs to two disks,
    so the solid count is the sum of per-disk counts.
    """
    rng = np.random.default_rng(seed)
    target = (1.0 - porosity) * N * N
    solid = np.zeros((N, N), dtype=np.uint8)
    cell = 2.0 * r_max + gap
    nc = max(1, int(math.ceil(N / cell)))
    grid: dict[tuple[int, int], list[int]] = {}
    cx_l: list[float] = []
    cy_l: list[float] = []
    r_l: list[float] = []
    count = 0
    attempts = 0
    batch = 4096
    lo_pad = margin
    while count < target and attempts < max_attempts:
        r = rng.uniform(r_min, r_max, size=batch)
        u = rng.uniform(0.0, 1.0, size=(batch, 2))
        for t in range(batch):
            attempts += 1
            rt = float(r[t])
            span = (N - 1) - 2.0 * (rt + lo_pad)
            if span <= 0.0:
                continue
            ci = lo_pad + rt + float(u[t, 0]) * span
            cj = lo_pad + rt + float(u[t, 1]) * span
            gi, gj = int(ci // cell), int(cj // cell)
            ok = True
            for di in (-1, 0, 1):
                for dj in (-1, 0, 1):
                    for k in grid.get((gi + di, gj + dj), ()):
                        dx = ci - cx_l[k]
                        dy = cj - cy_l[k]
                        if dx * dx + dy * dy < (rt + r_l[k] + gap) ** 2:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                continue
            i0, i1 = int(math.ceil(ci - rt)), int(math.floor(ci + rt))
            j0, j1 = int(math.ceil(cj - rt)), int(math.floor(cj + rt))
            ii = np.arange(i0, i1 + 1, dtype=np.float64)
            jj = np.arange(j0, j1 + 1, dtype=np.float64)
            inside = ((ii[None, :] - ci) ** 2 + (jj[:, None] - cj) ** 2) <= rt * rt
            solid[j0:j1 + 1, i0:i1 + 1] |= inside.astype(np.uint8)
            count += int(inside.sum())
            grid.setdefault((gi, gj), []).append(len(r_l))
            cx_l.append(ci)
            cy_l.append(cj)
            r_l.append(rt)
            if count >= target:
                break
    del nc
    centers = np.stack([np.asarray(cx_l), np.asarray(cy_l)], axis=1) if r_l else np.zeros((0, 2))
    return DiskPack(solid=solid, centers=centers, radii=np.asarray(r_l),
                    porosity=1.0 - count / float(N * N))


def wall_normals(pack: DiskPack) -> np.ndarray:
    """Unit outward normal of the fluid domain (pointing into the grain) at
    every fluid node next to a solid node, float32 [2, N, N] (x plane then
    y plane, zero elsewhere): the unit vector from the node towards the
    centre of the grain whose surface is nearest to it."""
    solid = pack.solid != 0
    N = solid.shape[0]
    out = np.zeros((2, N, N), np.float32)
    pad = np.pad(solid, 1)
    near = np.zeros_like(solid)
    for dj in (-1, 0, 1):
        for di in (-1, 0, 1):
            near |= pad[1 + dj:1 + dj + N, 1 + di:1 + di + N]
    jj, ii = np.nonzero(near & ~solid)
    if len(jj) == 0 or len(pack.radii) == 0:
        return out
    best = np.full(len(jj), np.inf)
    nx = np.zeros(len(jj))
    ny = np.zeros(len(jj))
    for (ci, cj), r in zip(pack.centers, pack.radii):
        dx, dy = ci - ii, cj - jj
        d = np.hypot(dx, dy)
        gap = d - r
        take = gap < best
        best = np.where(take, gap, best)
        nx = np.where(take, dx / d, nx)
        ny = np.where(take, dy / d, ny)
    out[0, jj, ii] = nx
    out[1, jj, ii] = ny
    return out


# ----------------------------------------------------------------------------
# divergence-free advection velocity from a seeded stream function
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class StreamFunction:
    """psi(x, y) = sum_m a_m sin(2 pi (p_m x + phi_m)) sin(2 pi (q_m y + chi_m))
    over the unit square x = X/L, y = Y/L; velocity = scale * (d psi/dY, -d psi/dX)."""
    a: np.ndarray
    p: np.ndarray
    q: np.ndarray
    phi: np.ndarray
    chi: np.ndarray
    L: float
    scale: float = 1.0

    def velocity(self, X: np.ndarray, Y: np.ndarray):
        x = np.asarray(X, dtype=np.float64) / self.L
        y = np.asarray(Y, dtype=np.float64) / self.L
        vx = np.zeros(np.broadcast(x, y).shape)
        vy = np.zeros_like(vx)
        tp = 2.0 * math.pi
        for a, p, q, ph, ch in zip(self.a, self.p, self.q, self.phi, self.chi):
            sx = np.sin(tp * (p * x + ph))
            cx = np.cos(tp * (p * x + ph))
            sy = np.sin(tp * (q * y + ch))
            cy = np.cos(tp * (q * y + ch))
            vx += a * sx * cy * (tp * q / self.L)
            vy -= a * cx * sy * (tp * p / self.L)
        return self.scale * vx, self.scale * vy


    def psi(self, X: np.ndarray, Y: np.ndarray):
        """scale * psi at (X, Y) (the velocity is its rotated gradient)."""
        x = np.asarray(X, dtype=np.float64) / self.L
        y = np.asarray(Y, dtype=np.float64) / self.L
        out = np.zeros(np.broadcast(x, y).shape)
        tp = 2.0 * math.pi
        for a, p, q, ph, ch in zip(self.a, self.p, self.q, self.phi, self.chi):
            out += a * np.sin(tp * (p * x + ph)) * np.sin(tp * (q * y + ch))
        return self.scale * out


def stream_function(seed: int, L: float, n_modes: int = 8, max_wavenumber: int = 4) -> StreamFunction:
    rng = np.random.default_rng(seed)
    return StreamFunction(a=rng.standard_normal(n_modes),
                          p=rng.integers(1, max_wavenumber + 1, size=n_modes).astype(np.float64),
                          q=rng.integers(1, max_wavenumber + 1, size=n_modes).astype(np.float64),
                          phi=rng.uniform(0.0, 1.0, size=n_modes),
                          chi=rng.uniform(0.0, 1.0, size=n_modes),
                          L=L)


# ----------------------------------------------------------------------------
# pore flow: the stream function damped to zero at the grain surfaces
# ----------------------------------------------------------------------------

def wall_factor(xs: np.ndarray, ys: np.ndarray, centers: np.ndarray, radii: np.ndarray, width: float):
    """phi = prod_k s(d_k / width) on the grid xs (columns) x ys (rows),
    where d_k is the distance to the surface of disk k (negative inside) and
    s(t) = 3t^2 - 2t^3 on [0, 1], 0 below and 1 above; returns phi and its
    gradient (dphi/dx, dphi/dy), each [len(ys), len(xs)].  Every factor is
    C^1 with zero slope at both ends, so phi is smooth where grains are
    close together, and phi and its gradient vanish on every disk surface."""
    xs = np.asarray(xs, dtype=np.float64)
    ys = np.asarray(ys, dtype=np.float64)
    phi = np.ones((len(ys), len(xs)))
    gx = np.zeros_like(phi)
    gy = np.zeros_like(phi)
    for (cx, cy), r in zip(np.asarray(centers, dtype=np.float64).reshape(-1, 2), np.asarray(radii, dtype=np.float64)):
        reach = r + width
        i0, i1 = np.searchsorted(xs, cx - reach), np.searchsorted(xs, cx + reach, side="right")
        j0, j1 = np.searchsorted(ys, cy - reach), np.searchsorted(ys, cy + reach, side="right")
        if i0 >= i1 or j0 >= j1:
            continue
        DX = xs[None, i0:i1] - cx
        DY = ys[j0:j1, None] - cy
        rho = np.hypot(DX, DY)
        t = np.clip((rho - r) / width, 0.0, 1.0)
        sk = t * t * (3.0 - 2.0 * t)
        dk = np.where((t > 0.0) & (t < 1.0), 6.0 * t * (1.0 - t) / width, 0.0)
        safe = np.where(rho > 0.0, rho, 1.0)
        box = np.s_[j0:j1, i0:i1]
        # product rule with the old phi, then phi *= s_k
        gx[box] = gx[box] * sk + phi[box] * dk * (DX / safe)
        gy[box] = gy[box] * sk + phi[box] * dk * (DY / safe)
        phi[box] *= sk
    return phi, gx, gy


@dataclasses.dataclass
class PoreFlow:
    """Velocity v = (d(psi phi)/dY, -d(psi phi)/dX): the stream function of
    ``sf`` times the wall factor of the grains (disk centres in domain
    coordinates).  Divergence-free, zero on and inside the grains, equal to
    the plain stream-function flow farther than ``width`` from every grain."""
    sf: StreamFunction
    centers: np.ndarray
    radii: np.ndarray
    width: float = 6.0

    def velocity_grid(self, xs: np.ndarray, ys: np.ndarray):
        Y, X = np.meshgrid(np.asarray(ys, float), np.asarray(xs, float), indexing="ij")
        phi, px, py = wall_factor(xs, ys, self.centers, self.radii, self.width)
        psi = self.sf.psi(X, Y)
        ux, uy = self.sf.velocity(X, Y)
        return phi * ux + psi * py, phi * uy - psi * px


# ----------------------------------------------------------------------------
# Gaussian pulse initial condition
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Pulse:
    xc: float   # centre, domain coordinates
    yc: float
    sigma: float

    def __call__(self, X, Y):
        return np.exp(-((X - self.xc) ** 2 + (Y - self.yc) ** 2) / (2.0 * self.sigma ** 2))


def gaussian_pulse(seed: int, L: float) -> Pulse:
    """Unit-peak Gaussian; centre ~ U[0.4, 0.6]^2 and sigma ~ U[0.05, 0.1] in
    unit-square units, scaled by L."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.4, 0.6, size=2)
    s = rng.uniform(0.05, 0.1)
    return Pulse(xc=float(c[0] * L), yc=float(c[1] * L), sigma=float(s * L))


def gaussian_hill_1d(x, t: float, phi: float = 0.1, sigma0: float = 1e-2, x0: float = 0.3, v: float = 1.0,
                     D: float = 1e-2) -> np.ndarray:
    """The advected, spreading Gaussian hill of mass phi on the real line
    (the 1-D example of Sec. 7.1): its initial condition at t = 0, and the
    closed-form solution the printed errors are measured against."""
    s2 = sigma0 ** 2 + 2.0 * D * t
    return phi / np.sqrt(2.0 * np.pi * s2) * np.exp(-(np.asarray(x, np.float64) - x0 - v * t) ** 2 / (2.0 * s2))


def random_populations(N: int, seed: int, lo: float = 0.2, hi: float = 1.0) -> np.ndarray:
    """Strictly positive random population field [9, N, N] (FP64) for
    single-sweep tests that start away from equilibrium."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(9, N, N))


def reaction_field(N: int, seed: int, k_max: float) -> np.ndarray:
    """Per-node first-order reaction rate, uniform in [0, k_max]."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, k_max, size=(N, N))
