"""Seeded synthetic initial conditions for the coupled phase-field / hydro LBM.

This module only builds initial fields (phi, u, p*) as float64 numpy arrays of
shape (nz, ny, nx) / (3, nz, ny, nx), x fastest.  It holds none of the method's
arithmetic; the same arrays are handed to the GPU library and to the CPU
oracle so both start from identical bits.

Shapes follow the paper's workloads: a droplet or bubble with the planar
equilibrium profile phi = phi_0 +- (phi_H - phi_L)/2 tanh(2 d / xi) across its
surface (Section 3.1), bubbles in a box with walls at the top and bottom
(Section 6.1), and a swarm of bubbles of random size (Section 6.2).
Random numbers come from numpy's PCG64 with a recorded seed.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict

import numpy as np

DEFAULT_SEED = 2020


@dataclass
class Setup:
    """One workload: grid, physical parameters and a recipe for the fields."""
    name: str
    nx: int
    ny: int
    nz: int
    walls_y: bool
    phi_L: float = 0.0
    phi_H: float = 1.0
    xi: float = 5.0
    mobility: float = 0.02
    sigma: float = 1e-4
    rho_L: float = 0.001
    rho_H: float = 1.0
    tau_L: float = 0.3
    tau_H: float = 0.03
    accel: tuple = (0.0, 0.0, 0.0)
    buoyancy_rho_ref: float = 0.0
    normal_eps: float = 1e-12
    density_literal: bool = False
    steps: int = 1000
    # field recipe
    kind: str = "bubble"          # "bubble" (light inside), "droplet" (heavy inside), "swarm", "uniform"
    radius: float = 16.0
    center: tuple = (64.0, 64.0, 64.0)
    noise: float = 0.0
    n_bubbles: int = 0
    d_range: tuple = (16.0, 32.0)
    seed: int = DEFAULT_SEED
    extra: dict = field(default_factory=dict)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def cells(self):
        return self.nx * self.ny * self.nz

    def physics(self) -> dict:
        """The parameters both sides take (names as in the C structs)."""
        return dict(nx=self.nx, ny=self.ny, nz=self.nz, walls_y=bool(self.walls_y),
                    phi_L=self.phi_L, phi_H=self.phi_H, xi=self.xi, mobility=self.mobility,
                    sigma=self.sigma, rho_L=self.rho_L, rho_H=self.rho_H,
                    tau_L=self.tau_L, tau_H=self.tau_H, accel=tuple(self.accel),
                    buoyancy_rho_ref=self.buoyancy_rho_ref, normal_eps=self.normal_eps,
                    density_literal=bool(self.density_literal))

    def with_grid(self, nx, ny, nz, **kw):
        d = asdict(self)
        d.update(nx=nx, ny=ny, nz=nz)
        d.update(kw)
        return Setup(**d)


def tau_from_dynamic_viscosity(mu: float, rho: float) -> float:
    """Model tau of nu = tau c_s^2 (dx = dt = 1) for a dynamic viscosity."""
    return 3.0 * mu / rho


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

def static_droplet(n: int = 32, R: float = 8.0, seed: int = DEFAULT_SEED, noise: float = 1e-6,
                   steps: int = 1000) -> Setup:
    """Static heavy droplet, fully periodic, 32^3, R = 8, xi = 4, M = 0.02,
    sigma = 1e-3, rho_H = 10, rho_L = 1, tau = 1 in both phases, no gravity,
    u = seeded uniform +-1e-6 noise made mean-free."""
    c = n / 2.0
    return Setup(name=f"static_droplet_{n}", nx=n, ny=n, nz=n, walls_y=False,
                 xi=4.0, mobility=0.02, sigma=1e-3, rho_L=1.0, rho_H=10.0,
                 tau_L=1.0, tau_H=1.0, steps=steps, kind="droplet", radius=R,
                 center=(c, c, c), noise=noise, seed=seed)


def rising_bubble(nx: int = 128, ny: int = 512, nz: int = 128, D: float = 32.0,
                  center=(64.0, 64.0, 64.0), g: float = 9.78e-7, steps: int = 20000) -> Setup:
    """Single rising bubble: y up, periodic x/z, walls at y = 0 and ny-1,
    rho_H = 1, rho_L = 0.001, mu_H = 0.01, mu_L = 1e-4, xi = 5, M = 0.02,
    sigma = 1e-4, gravity g along -y, u = 0, p* = 0.  Buoyancy is taken
    relative to the heavy fluid, F_b = (rho - rho_H) g (buoyancy_rho_ref =
    rho_H): between the walls this is the printed rho g less the heavy fluid's
    hydrostatic pressure."""
    return Setup(name=f"rising_bubble_{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, walls_y=True,
                 xi=5.0, mobility=0.02, sigma=1e-4, rho_L=0.001, rho_H=1.0,
                 tau_L=tau_from_dynamic_viscosity(1e-4, 0.001),
                 tau_H=tau_from_dynamic_viscosity(0.01, 1.0),
                 accel=(0.0, -g, 0.0), buoyancy_rho_ref=1.0, steps=steps, kind="bubble",
                 radius=D / 2.0, center=tuple(center))


def bubble_swarm(n: int = 512, n_bubbles: int = 200, d_range=(16.0, 32.0),
                 seed: int = DEFAULT_SEED, steps: int = 2000) -> Setup:
    """Bubble swarm: n^3, walls at y = 0 and n-1, rising-bubble physics,
    ``n_bubbles`` non-overlapping bubbles with diameters uniform in d_range
    at seeded uniform-random centres."""
    s = rising_bubble(n, n, n, steps=steps)
    s.name = f"bubble_swarm_{n}"
    s.kind = "swarm"
    s.n_bubbles = n_bubbles
    s.d_range = tuple(d_range)
    s.seed = seed
    return s


def surrogate_jump_bubble(steps: int = 40000) -> Setup:
    """Large rising bubble: 256 x 1024 x 256, D = 48 at (128, 256, 128),
    Eo = g rho_H D^2 / sigma = 10."""
    D, sigma, rho_H, Eo = 48.0, 1e-4, 1.0, 10.0
    g = Eo * sigma / (rho_H * D * D)
    s = rising_bubble(256, 1024, 256, D=D, center=(128.0, 256.0, 128.0), g=g, steps=steps)
    s.name = "rising_bubble_256x1024x256"
    return s


def drag_bubble(re_gr: float, eo: float = 30.0, D: float = 32.0, t_ref: float = 2000.0,
                grid=(256, 1024, 256), center=None) -> Setup:
    """The paper's single rising bubble for the drag coefficient (Sec. 6.1):
    256 x 1024 x 256 with walls at y = 0 and 1023, D = 32 at (128, 256, 128),
    density ratio 1000 and viscosity ratio 100, xi = 5, M = 0.04.  The
    dimensionless groups fix the lattice parameters once the reference time
    t_ref = sqrt(D/g) (in steps) is chosen: g = D / t_ref^2,
    Eo = g rho_H D^2 / sigma gives sigma, Re_Gr = rho_H sqrt(g D^3) / mu_H gives
    mu_H, and mu_L = mu_H / 100, rho_L = rho_H / 1000."""
    nx, ny, nz = grid
    rho_H, rho_L = 1.0, 1e-3
    g = D / (t_ref * t_ref)
    sigma = g * rho_H * D * D / eo
    mu_H = rho_H * np.sqrt(g * D ** 3) / re_gr
    mu_L = mu_H / 100.0
    c = center if center is not None else (nx / 2.0, ny / 4.0, nz / 2.0)
    s = Setup(name=f"drag_bubble_{nx}x{ny}x{nz}_Eo{eo:g}_Re{re_gr:g}", nx=nx, ny=ny, nz=nz, walls_y=True,
              xi=5.0, mobility=0.04, sigma=sigma, rho_L=rho_L, rho_H=rho_H,
              tau_L=tau_from_dynamic_viscosity(mu_L, rho_L), tau_H=tau_from_dynamic_viscosity(mu_H, rho_H),
              accel=(0.0, -g, 0.0), buoyancy_rho_ref=rho_H, steps=int(round(10 * t_ref)), kind="bubble",
              radius=D / 2.0, center=tuple(c))
    return s


def paper_benchmark_bubble(n: int = 260) -> Setup:
    """The paper's single-GPU benchmark: n^3 periodic, gas bubble R = 65 in
    the middle, rho 1 / 0.001, M = 0.02, xi = 5, sigma = 1e-4, tau = 0.03, no
    force, 200 steps."""
    c = n / 2.0
    return Setup(name=f"paper_bubble_{n}", nx=n, ny=n, nz=n, walls_y=False, xi=5.0,
                 mobility=0.02, sigma=1e-4, rho_L=0.001, rho_H=1.0, tau_L=0.03, tau_H=0.03,
                 steps=200, kind="bubble", radius=65.0 * n / 260.0, center=(c, c, c))


WORKLOADS = {
    "static_droplet_32": static_droplet,
    "rising_bubble_128x512x128": rising_bubble,
    "bubble_swarm_512": bubble_swarm,
    "rising_bubble_256x1024x256": surrogate_jump_bubble,
    "paper_bubble_260": paper_benchmark_bubble,
}


# ---------------------------------------------------------------------------
# field builders
# ---------------------------------------------------------------------------

def _axis(n):
    return np.arange(n, dtype=np.float64)


def _sphere_profile(setup: Setup, center, R, light_inside: bool, out=None):
    """phi of one sphere on the whole grid (distance without periodic images)."""
    z, y, x = np.meshgrid(_axis(setup.nz), _axis(setup.ny), _axis(setup.nx), indexing="ij")
    r = np.sqrt((x - center[0]) ** 2 + (y - center[1]) ** 2 + (z - center[2]) ** 2)
    half = 0.5 * (setup.phi_H - setup.phi_L)
    phi0 = 0.5 * (setup.phi_H + setup.phi_L)
    sgn = 1.0 if light_inside else -1.0
    return phi0 + sgn * half * np.tanh(2.0 * (r - R) / setup.xi)


def _swarm_centres(setup: Setup, rng):
    """Rejection-sample non-overlapping bubbles: |c_a - c_b| >= R_a + R_b + 2 xi
    (minimum image in x and z), and every bubble at least R + xi from the
    walls."""
    dmin, dmax = setup.d_range
    centres, radii = [], []
    tries = 0
    while len(centres) < setup.n_bubbles:
        tries += 1
        if tries > 200000:
            raise RuntimeError("could not place the requested bubbles")
        R = 0.5 * rng.uniform(dmin, dmax)
        lo = R + setup.xi + (1.0 if setup.walls_y else 0.0)
        hi_y = setup.ny - 1 - lo if setup.walls_y else setup.ny
        c = np.array([rng.uniform(0, setup.nx), rng.uniform(lo if setup.walls_y else 0, hi_y),
                      rng.uniform(0, setup.nz)])
        ok = True
        for c2, R2 in zip(centres, radii):
            d = c - c2
            d[0] -= setup.nx * round(d[0] / setup.nx)
            d[2] -= setup.nz * round(d[2] / setup.nz)
            if not setup.walls_y:
                d[1] -= setup.ny * round(d[1] / setup.ny)
            if np.sqrt((d * d).sum()) < R + R2 + 2.0 * setup.xi:
                ok = False
                break
        if ok:
            centres.append(c)
            radii.append(R)
    return np.array(centres), np.array(radii)


def _swarm_phi(setup: Setup, rng):
    """phi = min over bubbles of each bubble's profile, evaluated in a box of
    half-width R + 10 xi around each centre (beyond it the profile equals
    phi_H to double precision), minimum image in x and z."""
    centres, radii = _swarm_centres(setup, rng)
    phi = np.full(setup.shape, setup.phi_H, dtype=np.float64)
    half = 0.5 * (setup.phi_H - setup.phi_L)
    phi0 = 0.5 * (setup.phi_H + setup.phi_L)
    for c, R in zip(centres, radii):
        m = int(math.ceil(R + 10.0 * setup.xi))
        xs = np.arange(int(math.floor(c[0])) - m, int(math.floor(c[0])) + m + 2)
        zs = np.arange(int(math.floor(c[2])) - m, int(math.floor(c[2])) + m + 2)
        ys = np.arange(max(0, int(math.floor(c[1])) - m), min(setup.ny, int(math.floor(c[1])) + m + 2))
        xs = xs[: setup.nx]
        zs = zs[: setup.nz]
        Z, Y, X = np.meshgrid(zs.astype(np.float64), ys.astype(np.float64),
                              xs.astype(np.float64), indexing="ij")
        r = np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2)
        prof = phi0 + half * np.tanh(2.0 * (r - R) / setup.xi)
        iz = (zs % setup.nz)[:, None, None]
        iy = ys[None, :, None]
        ix = (xs % setup.nx)[None, None, :]
        sub = phi[iz, iy, ix]
        phi[iz, iy, ix] = np.minimum(sub, prof)
    return phi, centres, radii


def build_fields(setup: Setup):
    """Return (phi, u, pstar) float64 arrays for ``setup``.

    Wall rows (y = 0, ny-1 when walls_y) are set to zero in every field."""
    rng = np.random.Generator(np.random.PCG64(setup.seed))
    if setup.kind == "droplet":
        phi = _sphere_profile(setup, setup.center, setup.radius, light_inside=False)
    elif setup.kind == "bubble":
        phi = _sphere_profile(setup, setup.center, setup.radius, light_inside=True)
    elif setup.kind == "swarm":
        phi, centres, radii = _swarm_phi(setup, rng)
        setup.extra["centres"] = centres.tolist()
        setup.extra["radii"] = radii.tolist()
    elif setup.kind == "uniform":
        phi = np.full(setup.shape, setup.extra.get("phi", setup.phi_H), dtype=np.float64)
    else:
        raise ValueError(f"unknown field kind {setup.kind!r}")
    u = np.zeros((3,) + setup.shape, dtype=np.float64)
    if setup.noise > 0.0:
        u = setup.noise * (2.0 * rng.random((3,) + setup.shape) - 1.0)
    pstar = np.zeros(setup.shape, dtype=np.float64)
    if setup.walls_y:
        phi[:, 0, :] = 0.0
        phi[:, -1, :] = 0.0
        u[:, :, 0, :] = 0.0
        u[:, :, -1, :] = 0.0
    if setup.noise > 0.0:
        fluid = np.ones(setup.shape, dtype=bool)
        if setup.walls_y:
            fluid[:, 0, :] = False
            fluid[:, -1, :] = False
        for a in range(3):
            u[a][fluid] -= u[a][fluid].mean()
    return np.ascontiguousarray(phi), np.ascontiguousarray(u), pstar
