"""Dam-break, still-water column and free-blob layouts (seeded, FP64, host).

The paper's testbed is the gravity collapse of a water column in a tank
(Section 2, Fig. 2); its geometry is not given, so these layouts stand in for
it.  Conventions (all lengths in metres):

* Particles sit on a cubic lattice of spacing ``dp`` at ``(i + 1/2) dp``.
* Fluid: a block against the x = 0 and y = 0 walls and the floor, with seeded
  uniform jitter of +-``jitter * dp`` per coordinate.
* Boundary (dynamic boundary particles, Table 1): exact lattice points in two
  layers outside the tank interior ``[0, Lx] x [0, Ly] x [0, Lz]``; no lid.
* Boundary particles come first (ids ``0 .. nb-1``), fluid after them.
* Initial fluid density is hydrostatic for the Tait law (the reading used for
  the still-water state): ``rho = rho0 (1 + rho0 |g| (H - z) / B)^(1/gamma)``
  with ``B = c0^2 rho0 / gamma``; boundary density is ``rho0``.
* Domain box: ``[-2dp, Lx+2dp] x [-2dp, Ly+2dp] x [-2dp, 2 Lz]``; a particle
  outside it is excluded from the computation.

Only inputs are produced here.  Nothing in this module evaluates the SPH
kernel, the pair terms or the time integrator.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

SEED_BASE = 11103711


@dataclass(frozen=True)
class Physics:
    """Constants of one case (Table 1 formulation).

    ``h`` is the smoothing length, 1.2 sqrt(3) dp; the kernel support is ``2h``.
    ``c0`` = 10 sqrt(g H) for the column height H; ``eta2`` = 0.01 h^2 (the
    regulariser of the Monaghan term); ``mass`` = rho0 dp^3; ``cfl`` = 0.2.
    Corrective Verlet step every ``verlet_ns`` steps; ``bound_floor`` keeps
    boundary densities at or above rho0.
    ``kernel`` 0 = Wendland quintic, 1 = cubic spline.
    ``tensile_dp`` > 0 switches the tensile correction on, with that spacing
    in f = W(r)/W(dp); 0 = off.
    """

    dp: float
    h: float
    rho0: float
    gamma: float
    c0: float
    alpha: float
    eta2: float
    g: tuple
    mass: float
    cfl: float
    verlet_ns: int = 40
    bound_floor: int = 1
    kernel: int = 0
    tensile_dp: float = 0.0


def physics(dp: float, column_height: float = 0.2, alpha: float = 0.1,
            kernel: int = 0, gravity: float = 9.81, coef_h: float = 1.2) -> Physics:
    h = coef_h * math.sqrt(3.0) * dp
    c0 = 10.0 * math.sqrt(9.81 * column_height)
    return Physics(dp=dp, h=h, rho0=1000.0, gamma=7.0, c0=c0, alpha=alpha,
                   eta2=0.01 * h * h, g=(0.0, 0.0, -gravity),
                   mass=1000.0 * dp ** 3, cfl=0.2, kernel=kernel)


@dataclass
class Layout:
    """One particle set: FP64 arrays indexed by particle id."""

    name: str
    x: np.ndarray          # (n, 3) float64 positions
    v: np.ndarray          # (n, 3) float64 velocities
    rho: np.ndarray        # (n,)   float64 densities
    nb: int                # ids [0, nb) are boundary particles
    phys: Physics
    lo: np.ndarray         # (3,) domain lower corner
    hi: np.ndarray         # (3,) domain upper corner
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def nf(self) -> int:
        return self.n - self.nb

    def copy(self) -> "Layout":
        return replace(self, x=self.x.copy(), v=self.v.copy(), rho=self.rho.copy(),
                       meta=dict(self.meta))


@dataclass(frozen=True)
class Case:
    """A named configuration: layout recipe plus run settings."""

    name: str
    dp: float
    steps: int
    description: str


def cell_grid(layout: Layout, nsub: int = 1):
    """Cell grid covering the domain: cells of side ``2h/nsub`` (slightly
    enlarged by 2^-20 so that FP32 rounding never puts a pair inside the
    support but outside the (2 nsub + 1)^3 stencil).

    Returns ``(origin[3], cell, nc[3])`` with cells ordered X fastest, then Y,
    then Z (Section 4.4).
    """
    if nsub not in (1, 2):
        raise ValueError("nsub must be 1 or 2")
    cell = 2.0 * layout.phys.h / nsub * (1.0 + 2.0 ** -20)
    origin = np.asarray(layout.lo, dtype=np.float64).copy()
    nc = [int(math.ceil((layout.hi[i] - layout.lo[i]) / cell)) for i in range(3)]
    return origin, cell, nc


def _lattice(ix, iy, iz, dp):
    """Lattice points (i+1/2)dp for the index ranges, X fastest."""
    gz, gy, gx = np.meshgrid(np.arange(*iz), np.arange(*iy), np.arange(*ix), indexing="ij")
    pts = np.empty((gx.size, 3), dtype=np.float64)
    pts[:, 0] = (gx.ravel() + 0.5) * dp
    pts[:, 1] = (gy.ravel() + 0.5) * dp
    pts[:, 2] = (gz.ravel() + 0.5) * dp
    return pts


def _tank_walls(nx, ny, nz, dp, layers=2):
    """Two lattice layers outside the interior [0,nx)x[0,ny)x[0,nz), open top.

    Built as disjoint slabs: floor (full outer x/y extent), two x-walls
    (full outer y extent), two y-walls (interior x extent).
    """
    L = layers
    slabs = [
        _lattice((-L, nx + L), (-L, ny + L), (-L, 0), dp),          # floor
        _lattice((-L, 0), (-L, ny + L), (0, nz), dp),               # x-low wall
        _lattice((nx, nx + L), (-L, ny + L), (0, nz), dp),          # x-high wall
        _lattice((0, nx), (-L, 0), (0, nz), dp),                    # y-low wall
        _lattice((0, nx), (ny, ny + L), (0, nz), dp),               # y-high wall
    ]
    return np.concatenate(slabs, axis=0)


def dam_break(dp: float, seed: int, fluid=(0.2, 0.2, 0.2), tank=(0.8, 0.4, 0.4),
              jitter: float = 0.05, vel_sigma: float = 0.0, vel_seed: int | None = None,
              alpha: float = 0.1, kernel: int = 0, name: str = "dam_break") -> Layout:
    """Fluid block in the corner of an open tank of dynamic boundary particles."""
    nfx, nfy, nfz = (int(round(f / dp)) for f in fluid)
    ntx, nty, ntz = (int(round(t / dp)) for t in tank)
    if not (nfx <= ntx and nfy <= nty and nfz <= ntz):
        raise ValueError("fluid block larger than the tank")
    H = nfz * dp
    ph = physics(dp, column_height=H, alpha=alpha, kernel=kernel)

    bnd = _tank_walls(ntx, nty, ntz, dp)
    flu = _lattice((0, nfx), (0, nfy), (0, nfz), dp)
    if jitter:
        rng = np.random.default_rng(seed)
        flu += rng.uniform(-jitter * dp, jitter * dp, size=flu.shape)

    x = np.concatenate([bnd, flu], axis=0)
    nb = bnd.shape[0]
    n = x.shape[0]
    v = np.zeros((n, 3), dtype=np.float64)
    if vel_sigma:
        vrng = np.random.default_rng(seed if vel_seed is None else vel_seed)
        v[nb:] = vrng.normal(0.0, vel_sigma, size=(n - nb, 3))
    rho = np.full(n, ph.rho0, dtype=np.float64)
    B = ph.c0 ** 2 * ph.rho0 / ph.gamma
    depth = H - x[nb:, 2]
    rho[nb:] = ph.rho0 * np.power(1.0 + ph.rho0 * abs(ph.g[2]) * depth / B, 1.0 / ph.gamma)

    lo = np.array([-2 * dp, -2 * dp, -2 * dp])
    hi = np.array([ntx * dp + 2 * dp, nty * dp + 2 * dp, 2.0 * ntz * dp])
    return Layout(name=name, x=x, v=v, rho=rho, nb=nb, phys=ph, lo=lo, hi=hi,
                  meta={"dp": dp, "seed": seed, "fluid": tuple(fluid), "tank": tuple(tank),
                        "jitter": jitter, "vel_sigma": vel_sigma, "H": H})


def column(dp: float = 0.01, seed: int = SEED_BASE + 7, jitter: float = 0.0) -> Layout:
    """Still-water column: 0.1 x 0.1 x 0.2 m of fluid filling a 2-layer box."""
    return dam_break(dp, seed, fluid=(0.1, 0.1, 0.2), tank=(0.1, 0.1, 0.2),
                     jitter=jitter, name="column")


def blob(n_side: int, dp: float, seed: int, vel_sigma: float = 0.5, jitter: float = 0.2,
         gravity: bool = False, alpha: float = 0.1, rho_sigma: float = 5.0) -> Layout:
    """Free fluid cube (no boundaries), jittered, random velocities and
    densities; gravity off by default.  Used for conservation invariants."""
    rng = np.random.default_rng(seed)
    x = _lattice((0, n_side), (0, n_side), (0, n_side), dp)
    x += rng.uniform(-jitter * dp, jitter * dp, size=x.shape)
    x += 0.5  # keep the blob well inside its domain box
    n = x.shape[0]
    v = rng.normal(0.0, vel_sigma, size=(n, 3))
    ph = physics(dp, alpha=alpha, gravity=9.81 if gravity else 0.0)
    rho = ph.rho0 + rng.normal(0.0, rho_sigma, size=n)
    lo = np.array([0.5 - 3 * dp] * 3)
    hi = np.array([0.5 + (n_side + 3) * dp] * 3)
    return Layout(name="blob", x=x, v=v, rho=rho, nb=0, phys=ph, lo=lo, hi=hi,
                  meta={"dp": dp, "seed": seed, "n_side": n_side})


def refine(x_fluid, v_fluid, rho_fluid, dp: float, factor: int = 8, seed: int = SEED_BASE + 3,
           jitter: float = 0.05, tank=(0.8, 0.4, 0.4), alpha: float = 0.1, kernel: int = 0,
           name: str = "refined") -> Layout:
    """Clustered layout from a coarse fluid state (e.g. a dam-break snapshot):
    every fluid particle becomes ``factor^3`` children on a sub-lattice of
    spacing ``dp/factor`` centred on it, inheriting its velocity and density,
    with seeded uniform jitter of +-``jitter`` times the new spacing; the tank
    walls are regenerated at the new spacing.  Parent cubes overlap or leave
    gaps wherever the coarse particles were not on their lattice, which gives
    uneven density.  The domain box is the coarse case's (2 coarse spacings
    around the tank, twice its height), the box the coarse state lived in, so
    children of particles near a wall stay inside it.  Only the positions are
    built here: no kernel, pair term or integrator is evaluated."""
    x_fluid = np.asarray(x_fluid, dtype=np.float64).reshape(-1, 3)
    v_fluid = np.asarray(v_fluid, dtype=np.float64).reshape(-1, 3)
    rho_fluid = np.asarray(rho_fluid, dtype=np.float64).ravel()
    d = dp / factor
    sub = (np.arange(factor) + 0.5) * d - 0.5 * dp            # child offsets from the parent
    gz, gy, gx = np.meshgrid(sub, sub, sub, indexing="ij")
    off = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1)  # X fastest
    m = off.shape[0]
    flu = (x_fluid[:, None, :] + off[None, :, :]).reshape(-1, 3)
    if jitter:
        rng = np.random.default_rng(seed)
        flu += rng.uniform(-jitter * d, jitter * d, size=flu.shape)
    ntx, nty, ntz = (int(round(t / d)) for t in tank)
    bnd = _tank_walls(ntx, nty, ntz, d)
    ph = physics(d, alpha=alpha, kernel=kernel)
    x = np.concatenate([bnd, flu], axis=0)
    nb = bnd.shape[0]
    n = x.shape[0]
    v = np.zeros((n, 3), dtype=np.float64)
    v[nb:] = np.repeat(v_fluid, m, axis=0)
    rho = np.full(n, ph.rho0, dtype=np.float64)
    rho[nb:] = np.repeat(rho_fluid, m)
    lo = np.array([-2 * dp, -2 * dp, -2 * dp])
    hi = np.array([ntx * d + 2 * dp, nty * d + 2 * dp, 2.0 * ntz * d])
    return Layout(name=name, x=x, v=v, rho=rho, nb=nb, phys=ph, lo=lo, hi=hi,
                  meta={"dp": d, "seed": seed, "factor": factor, "parents": x_fluid.shape[0]})


CASES = {
    "dam_break_8k": Case("dam_break_8k", 0.01, 100,
                         "3D dam break, 8,000 fluid + 27,232 boundary particles (dp = 0.01 m)"),
    "dam_break_1m": Case("dam_break_1m", 0.002, 1000,
                         "3D dam break, 1,000,000 fluid + 648,032 boundary particles "
                         "(dp = 0.002 m)"),
    "dam_break_64k": Case("dam_break_64k", 0.005, 200,
                          "3D dam break, 64,000 fluid + 105,632 boundary particles (dp = 0.005 m), "
                          "seeded N(0, 0.01^2) initial fluid velocity"),
    "dam_break_20m": Case("dam_break_20m", 0.2 / 272, 200,
                          "3D dam break, 20,123,648 fluid + 4,756,768 boundary particles "
                          "(dp = 0.2/272 m)"),
}

# jitter seed offsets from SEED_BASE, and the initial-velocity seed of the
# 64k case
_SEED = {"dam_break_8k": 1, "dam_break_1m": 2, "dam_break_64k": 4, "dam_break_20m": 5}
VEL_SEED_64K = SEED_BASE + 40
CLUSTER_SEED = SEED_BASE + 3   # jitter of the refined (clustered) layout


def named_case(name: str) -> Layout:
    """Layout of a named workload, seeded from ``SEED_BASE`` plus its offset."""
    c = CASES[name]
    seed = SEED_BASE + _SEED[name]
    if name == "dam_break_64k":
        return dam_break(c.dp, seed, vel_sigma=0.01, vel_seed=VEL_SEED_64K, name=name)
    return dam_break(c.dp, seed, name=name)
