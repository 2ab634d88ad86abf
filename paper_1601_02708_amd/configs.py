"""Run descriptors for the hybrid FEM/LBM workloads and the seeded problem
arrays they expand to.

Three workloads are defined, all in lattice units (fine spacing 1, fine
step 1, coarse step = eta):

* ``small``  -- 64^2 lattice, 16^2 bilinear mesh, uniform velocity
  (0.05, 0), D = 1e-2, no reaction, 4 substeps x 100 coarse steps x 2
  Schwarz iterations.  Correctness workload.
* ``pore2048`` -- 2048^2 lattice with random disks (porosity 0.6), a
  seeded 8-mode stream-function velocity damped to zero within 6 lattice
  units of the grain surfaces (divergence-free, no flow into the solids;
  max |v| = 0.05 over fluid nodes), D = 5e-3, first-order reaction
  k = 1e-4, 128^2 mesh,
  10 substeps x 200 coarse steps x 2 Schwarz iterations.  Throughput
  workload.
* ``pore4096`` -- the same generators at 4096^2 with D = 1e-2, no reaction,
  16^2 mesh, 4 substeps x 100 coarse steps x 2 Schwarz iterations.
  Precision workload.
* ``diff512`` -- the differentiation workload: 512^2 lattice with the
  pore2048 generators, 64^2 mesh, D = 5e-3, 10 substeps x 200 coarse steps
  (2000 fine steps) x 1 Schwarz iteration, a per-node fine reaction rate
  U[0, 2e-4] (the coarse model takes its mean 1e-4), an inlet: the edge
  x = 0 held at 1, the other three edges with the natural condition.
* ``dissolve4096`` -- dissolving solids: the same generators at 4096^2 with
  porosity 0.5, D = 1e-2, bulk reaction k = 1e-4, 256^2 mesh, 20 substeps x
  500 coarse steps x 2 Schwarz iterations; a surface reaction of rate
  kappa_s = 0.01 towards c_sat = 1 at every fluid-solid link and a seeded
  mass in U[0.5, 1.0] per solid node (``solid_mass``).

The descriptors carry the diffusion coefficient D only (plus an optional
relaxation-time override): the solvers derive the BGK relaxation time from
D themselves (Sec. 4.1).  The outer boundary of the coarse domain is
Dirichlet 0 on all four edges, and the initial condition is the seeded
Gaussian pulse on both grids.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from . import inputs


@dataclasses.dataclass(frozen=True)
class HybridConfig:
    name: str
    N: int                      # fine nodes per side
    M: int                      # coarse elements per side
    D: float                    # diffusion coefficient (lattice units)
    eta: int                    # fine substeps per coarse step
    steps: int                  # coarse steps
    max_iter: int               # Schwarz iterations per coarse step
    k: float = 0.0              # uniform first-order reaction rate (per lattice step)
    porosity: Optional[float] = None     # None: no solids
    velocity: str = "uniform"            # "uniform" or "stream"
    v_uniform: tuple = (0.05, 0.0)
    v_max: float = 0.05
    wall_width: float = 6.0              # lattice units over which the flow vanishes at grains
    overlap_elems: int = 1      # overlap width in coarse elements
    supg: int = 1
    bc_clamp: int = 0           # maxent Dirichlet: 0 closed form as printed, 1 clamp at 0
    seed: int = 0
    tau: Optional[float] = None  # BGK relaxation time override; None: each solver derives it from D
    # dissolving solids (kappa_s = 0: fixed solids)
    kappa_s: float = 0.0        # surface reaction rate at fluid-solid links
    c_sat: float = 1.0          # concentration the surface reaction drives towards
    mass_range: tuple = (0.5, 1.0)   # per-solid-node mass, uniform
    # outer edges (0: x = 0, 1: x = L, 2: y = 0, 3: y = L): bit e set = the
    # natural condition (zero diffusive flux); the others Dirichlet at
    # outer_value
    outer_natural: int = 0
    outer_value: float = 0.0
    k_field_max: Optional[float] = None   # per-node fine rate U[0, k_field_max] (seeded); None: uniform k

    @property
    def L(self) -> float:
        return inputs.domain_side(self.N)

    def replace(self, **kw) -> "HybridConfig":
        return dataclasses.replace(self, **kw)


SMALL = HybridConfig(name="small", N=64, M=16, D=1e-2, eta=4, steps=100, max_iter=2,
                     velocity="uniform", v_uniform=(0.05, 0.0))
PORE2048 = HybridConfig(name="pore2048", N=2048, M=128, D=5e-3, eta=10, steps=200,
                        max_iter=2, k=1e-4, porosity=0.6, velocity="stream")
PORE4096 = HybridConfig(name="pore4096", N=4096, M=16, D=1e-2, eta=4, steps=100,
                        max_iter=2, k=0.0, porosity=0.6, velocity="stream")

DIFF512 = HybridConfig(name="diff512", N=512, M=64, D=5e-3, eta=10, steps=200, max_iter=1, k=1e-4, porosity=0.6,
                       velocity="stream", outer_natural=14, outer_value=1.0, k_field_max=2e-4)
DISSOLVE4096 = HybridConfig(name="dissolve4096", N=4096, M=256, D=1e-2, eta=20, steps=500,
                            max_iter=2, k=1e-4, porosity=0.5, velocity="stream", kappa_s=0.01, c_sat=1.0)

CONFIGS = {c.name: c for c in (SMALL, PORE2048, PORE4096, DIFF512, DISSOLVE4096)}


def solid_mass(cfg: HybridConfig, solid: np.ndarray) -> np.ndarray:
    """Seeded mass per solid node, uniform in cfg.mass_range (0 at fluid
    nodes), float64 [N, N]."""
    rng = np.random.default_rng(cfg.seed + 3000)
    lo, hi = cfg.mass_range
    return np.where(np.asarray(solid) != 0, rng.uniform(lo, hi, solid.shape), 0.0)


@dataclasses.dataclass
class Problem:
    """Host arrays of one seeded workload (shared by oracle and GPU path)."""
    cfg: HybridConfig
    solid: np.ndarray        # uint8 [N, N]
    vx: np.ndarray           # float32 [N, N] fine velocity (zero in solids)
    vy: np.ndarray
    vc: np.ndarray           # float64 [(M+1)^2, 2] coarse nodal velocity
    u0_fine: np.ndarray      # float64 [N, N]
    u0_coarse: np.ndarray    # float64 [(M+1)^2]
    porosity: float
    x0: float
    y0: float
    L: float
    k_field: Optional[np.ndarray] = None    # float64 [N, N] per-node fine rate, or None (uniform cfg.k)
    pack: Optional[inputs.DiskPack] = None   # the grains (patch lattice coordinates), or None


def build_problem(cfg: HybridConfig) -> Problem:
    N, M = cfg.N, cfg.M
    L = cfg.L
    x0 = inputs.patch_origin(N)
    X, Y = inputs.fine_coords(N)
    XC, YC = inputs.coarse_coords(M, L)

    if cfg.porosity is not None:
        pack = inputs.random_disks(N, cfg.porosity, seed=cfg.seed + 1000)
        solid = pack.solid
        porosity = pack.porosity
    else:
        pack = None
        solid = np.zeros((N, N), dtype=np.uint8)
        porosity = 1.0

    if cfg.velocity == "uniform":
        vx64 = np.full((N, N), cfg.v_uniform[0])
        vy64 = np.full((N, N), cfg.v_uniform[1])
        vc = np.empty(((M + 1) * (M + 1), 2))
        vc[:, 0] = cfg.v_uniform[0]
        vc[:, 1] = cfg.v_uniform[1]
    elif cfg.velocity == "stream":
        # stream function damped to zero at the grain surfaces (no flow into
        # the solids), scaled to max |v| = v_max over the fluid nodes
        sf = inputs.stream_function(cfg.seed + 2000, L)
        centers = pack.centers + x0 if porosity < 1.0 else np.zeros((0, 2))
        radii = pack.radii if porosity < 1.0 else np.zeros(0)
        flow = inputs.PoreFlow(sf, centers, radii, cfg.wall_width)
        fine_ax = x0 + np.arange(N, dtype=np.float64)
        coarse_ax = np.arange(M + 1, dtype=np.float64) * (L / M)
        vx64, vy64 = flow.velocity_grid(fine_ax, fine_ax)
        fluid = solid == 0
        vmax = float(np.sqrt(vx64 ** 2 + vy64 ** 2)[fluid].max())
        sf.scale = cfg.v_max / vmax
        vx64, vy64 = flow.velocity_grid(fine_ax, fine_ax)
        cvx, cvy = flow.velocity_grid(coarse_ax, coarse_ax)
        vc = np.stack([cvx.ravel(), cvy.ravel()], axis=1)
    else:
        raise ValueError(cfg.velocity)

    vx = vx64.astype(np.float32)
    vy = vy64.astype(np.float32)
    vx[solid != 0] = 0.0
    vy[solid != 0] = 0.0

    pulse = inputs.gaussian_pulse(cfg.seed, L)
    u0_fine = pulse(X, Y)
    u0_fine[solid != 0] = 0.0
    u0_coarse = pulse(XC, YC).ravel()
    k_field = None if cfg.k_field_max is None else inputs.reaction_field(N, cfg.seed + 4000, cfg.k_field_max)
    return Problem(cfg=cfg, solid=solid, vx=vx, vy=vy, vc=np.ascontiguousarray(vc), k_field=k_field,
                   u0_fine=u0_fine, u0_coarse=u0_coarse, porosity=porosity,
                   x0=x0, y0=x0, L=L, pack=pack)


# ----------------------------------------------------------------------------
# several fine patches in one coarse domain (Algorithm 2)
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Patch:
    """One fine lattice patch: N x N nodes, node (0, 0) at domain point
    (x0, y0); host arrays as in Problem."""
    N: int
    x0: float
    y0: float
    solid: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    u0_fine: np.ndarray


@dataclasses.dataclass
class MultiProblem:
    """A coarse mesh over [0, L]^2 with several disjoint fine patches."""
    M: int
    L: float
    D: float
    k: float
    eta: int
    max_iter: int
    supg: int
    overlap_elems: int
    bc_clamp: int
    vc: np.ndarray            # [(M+1)^2, 2] coarse nodal velocity
    u0_coarse: np.ndarray     # [(M+1)^2]
    patches: list


def build_multi(N: int, M: int, L: float, origins, D: float = 1e-2, k: float = 0.0, eta: int = 4,
                max_iter: int = 2, velocity=(0.05, 0.0), pulse=None, porosity=None, seed: int = 0) -> MultiProblem:
    """Fine patches of N x N nodes at the given domain origins, uniform
    velocity, the seeded Gaussian pulse (or the given one) as initial
    condition on every grid, random disks per patch at the given porosity
    (None: no solids)."""
    pulse = inputs.gaussian_pulse(seed, L) if pulse is None else pulse
    XC, YC = inputs.coarse_coords(M, L)
    vc = np.empty(((M + 1) * (M + 1), 2))
    vc[:, 0], vc[:, 1] = velocity
    patches = []
    for p, (x0, y0) in enumerate(origins):
        ax = np.arange(N, dtype=np.float64)
        Y, X = np.meshgrid(y0 + ax, x0 + ax, indexing="ij")
        if porosity is None:
            solid = np.zeros((N, N), np.uint8)
        else:
            solid = inputs.random_disks(N, porosity, seed=seed + 1000 + p, r_min=2, r_max=5).solid
        vx = np.full((N, N), velocity[0], np.float32)
        vy = np.full((N, N), velocity[1], np.float32)
        vx[solid != 0] = 0.0
        vy[solid != 0] = 0.0
        u0 = pulse(X, Y)
        u0[solid != 0] = 0.0
        patches.append(Patch(N=N, x0=float(x0), y0=float(y0), solid=solid, vx=vx, vy=vy, u0_fine=u0))
    return MultiProblem(M=M, L=float(L), D=D, k=k, eta=eta, max_iter=max_iter, supg=1, overlap_elems=1,
                        bc_clamp=0, vc=vc, u0_coarse=pulse(XC, YC).ravel(), patches=patches)
