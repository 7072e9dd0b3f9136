"""Pins of the whole oracle time step against physics the paper's model
must reproduce: exact conservation of sum(phi), the planar equilibrium
profile, Laplace's law, exact Poiseuille flow, layered Poiseuille flow
with variable viscosity (needs the viscous force), hydrostatics across a
density jump (needs the pressure force) and Galilean advection of an
interface.  None of the expected values comes from the oracle itself.
"""
import numpy as np
import pytest
from scipy.integrate import cumulative_trapezoid

from oracle import oracle as orc
from paper_2012_06144_amd import inputs

EPS64 = np.finfo(np.float64).eps


def _params(setup):
    return orc.Params(**setup.physics())


@pytest.fixture(scope="module")
def droplet_run():
    """Static droplet, 32^3 periodic, R = 8, xi = 4, sigma = 1e-3, rho 10/1,
    tau = 1, seeded +-1e-6 velocity noise, 1000 steps."""
    s = inputs.static_droplet()
    phi, u, ps = inputs.build_fields(s)
    o = orc.Oracle(_params(s))
    o.init(phi, u, ps)
    st0 = o.stats()
    o.step(s.steps)
    return s, o, st0, o.stats()


def test_mass_conserved_periodic(droplet_run):
    """P3: sum(phi) is conserved; the only change allowed is rounding, at
    most a few ulps per step relative to the total."""
    s, o, st0, st1 = droplet_run
    rel = abs(st1["mass"] - st0["mass"]) / st0["mass"]
    assert rel <= 4 * EPS64 * s.steps


def test_laplace_law(droplet_run):
    """P8: pressure jump across the droplet surface, p = p* rho cs^2 (Section
    3.2), equals 2 sigma / R within 5 %, R taken from the droplet volume."""
    s, o, st0, st1 = droplet_run
    p = o.pressure()
    n = s.nx
    z, y, x = np.meshgrid(*[np.arange(float(n))] * 3, indexing="ij")
    r = np.sqrt((x - 16) ** 2 + (y - 16) ** 2 + (z - 16) ** 2)
    p_in = p[r <= 2].mean()
    p_out = p[r >= s.radius + 1.5 * s.xi].mean()
    _, _, phi, _ = o.state()
    R_eff = (3 * phi.sum() / (4 * np.pi)) ** (1.0 / 3.0)
    ratio = (p_in - p_out) / (2 * s.sigma / R_eff)
    assert abs(ratio - 1.0) < 0.05, ratio
    assert abs((p_in - p_out) / (2 * s.sigma / s.radius) - 1.0) < 0.10


@pytest.mark.parametrize("R", [8.0, 16.0])
def test_laplace_law_cylinder(R):
    """P8 in two dimensions: a periodic column of heavy fluid (nz = 1) has the
    pressure jump sigma / R of a cylinder, half the sphere's 2 sigma / R.
    Within 3 % at xi = 4 for R = 8 and 16 (measured 0.03 %, 2.2 % at R = 12,
    2.5 % at 16, 2.0 % at 24: the error tends to the discretisation error of
    a xi = 4 interface as R grows; at fixed R/xi = 2 it tends instead to the
    diffuse interface's own O((xi/R)^2) correction, +3 % at R = 16, xi = 8)."""
    n, xi = int(4 * R), 4.0
    P = orc.Params(nx=n, ny=n, nz=1, xi=xi, mobility=0.02, sigma=1e-3, rho_L=1.0, rho_H=10.0,
                   tau_L=1.0, tau_H=1.0)
    y, x = np.meshgrid(np.arange(float(n)), np.arange(float(n)), indexing="ij")
    r = np.sqrt((x - n / 2) ** 2 + (y - n / 2) ** 2)
    o = orc.Oracle(P)
    o.init((0.5 + 0.5 * np.tanh(2 * (R - r) / xi)).reshape(1, n, n), np.zeros((3, 1, n, n)), np.zeros((1, n, n)))
    o.step(3000)
    p = o.pressure()[0]
    _, _, ph, _ = o.state()
    R_eff = np.sqrt(ph.sum() / np.pi)
    ratio = (p[r <= 2].mean() - p[r >= R + 1.5 * xi].mean()) / (P.sigma / R_eff)
    assert abs(ratio - 1.0) < 0.03, ratio


def test_static_droplet_stays_at_rest(droplet_run):
    """P9: the droplet does not move: spurious currents stay far below the
    capillary velocity sigma/mu and the centroid drifts by < 1e-3 cells."""
    s, o, st0, st1 = droplet_run
    mu = s.rho_H * s.tau_H / 3.0
    assert st1["max_speed"] < 1e-2 * s.sigma / mu
    drift = np.abs(np.array(st1["centroid"]) - np.array(st0["centroid"])).max()
    assert drift < 1e-3


def _circular_centre(phi):
    """Periodic centre of mass of phi about the box centre, from the phase
    of the first Fourier mode along each axis (invariant under wrap)."""
    out = []
    for ax_sum, L in ((2, phi.shape[2]), (1, phi.shape[1]), (0, phi.shape[0])):
        w = phi.sum(axis=tuple(a for a in range(3) if a != ax_sum))
        k = 2 * np.pi / L
        x = np.arange(L) - L / 2
        out.append(np.arctan2((w * np.sin(k * x)).sum(), (w * np.cos(k * x)).sum()) / k)
    return np.array(out)


def test_symmetric_droplet_centroid_fixed():
    """P9: a noise-free droplet centred on a node of a symmetric periodic box
    stays put (< 1e-3 cells in 300 steps).  It is not fixed to rounding:
    at the droplet centre grad(phi) = 0 while theta > 0, so the direction of
    the counter-flux theta n is set by rounding there; the offset this
    leaves is ~1e-4 cells for R = 6, xi = 3."""
    s = inputs.static_droplet(n=24, R=6.0, noise=0.0, steps=300)
    s.xi = 3.0
    phi, u, ps = inputs.build_fields(s)
    o = orc.Oracle(_params(s))
    o.init(phi, u, ps)
    c0 = _circular_centre(phi)
    assert np.abs(c0).max() < 1e-12
    o.step(s.steps)
    _, _, ph, _ = o.state()
    assert np.abs(_circular_centre(ph) - c0).max() < 1e-3


def test_mass_conserved_with_walls():
    """P3 with walls: halfway bounce-back of h keeps sum(phi) exact while a
    bubble rises under gravity between the y walls."""
    s = inputs.rising_bubble(16, 40, 16, D=10.0, center=(8.0, 14.0, 8.0), g=2e-5)
    phi, u, ps = inputs.build_fields(s)
    o = orc.Oracle(_params(s))
    o.init(phi, u, ps)
    st0 = o.stats()
    o.step(400)
    st1 = o.stats()
    rel = abs(st1["mass"] - st0["mass"]) / st0["mass"]
    assert rel <= 4 * EPS64 * 400
    assert st1["centroid"][1] > st0["centroid"][1] + 0.05   # it rises
    assert st1["rise_velocity"] > 0


def _flat_profile(nx, xi):
    x = np.arange(nx, dtype=float)
    a, b = nx / 4 - 0.5, 3 * nx / 4 - 0.5
    return np.minimum(0.5 + 0.5 * np.tanh(2 * (x - a) / xi), 0.5 + 0.5 * np.tanh(2 * (b - x) / xi))


@pytest.mark.parametrize("start", ["tanh", "step"])
def test_flat_interface_profile(start):
    """P7: a slab of heavy fluid relaxes to (or stays at) the planar
    equilibrium profile phi_0 + (phi_H - phi_L)/2 tanh(2 x / xi) of Section
    3.1; the measured width is xi."""
    nx, xi = 64, 4.0
    P = orc.Params(nx=nx, ny=4, nz=4, xi=xi, mobility=0.02, sigma=1e-3,
                   rho_L=1.0, rho_H=10.0, tau_L=1.0, tau_H=1.0)
    prof = _flat_profile(nx, xi)
    x = np.arange(nx, dtype=float)
    phi0 = prof if start == "tanh" else np.where((x > nx / 4 - 0.5) & (x < 3 * nx / 4 - 0.5), 1.0, 0.0)
    phi = np.broadcast_to(phi0, (4, 4, nx)).copy()
    o = orc.Oracle(P)
    o.init(phi, np.zeros((3, 4, 4, nx)), np.zeros((4, 4, nx)))
    o.step(3000)
    st = o.stats()
    _, _, ph, _ = o.state()
    # the stationary discrete profile deviates from tanh by 5.27e-3 at xi = 4
    # (second order in 1/xi: test_flat_interface_converges_to_tanh)
    assert np.abs(ph[0, 0] - prof).max() < 6e-3
    assert abs(st["xi_eff"] / xi - 1.0) < 1e-2
    assert np.abs(ph - ph[0:1, 0:1, :]).max() < 1e-14   # stays planar


def test_flat_interface_converges_to_tanh():
    """P7 under refinement: doubling the interface width (and the slab) cuts
    the stationary profile's deviation from the tanh of Section 3.1 by about
    4 (measured 5.27e-3 at xi = 4, 1.50e-3 at xi = 8, 3.9e-4 at xi = 16):
    the discrete equilibrium converges to it at second order in 1/xi."""
    dev = []
    for xi in (4.0, 8.0):
        nx = int(16 * xi)
        P = orc.Params(nx=nx, ny=1, nz=1, xi=xi, mobility=0.02, sigma=1e-3,
                       rho_L=1.0, rho_H=10.0, tau_L=1.0, tau_H=1.0)
        prof = _flat_profile(nx, xi)
        o = orc.Oracle(P)
        o.init(prof.reshape(1, 1, nx).copy(), np.zeros((3, 1, 1, nx)), np.zeros((1, 1, nx)))
        o.step(int(1000 * xi))
        _, _, ph, _ = o.state()
        dev.append(np.abs(ph[0, 0] - prof).max())
    assert dev[1] < 1.6e-3
    assert dev[0] / dev[1] > 3.3, dev


def _channel(ny, tau, a, rho=1.0):
    P = orc.Params(nx=1, ny=ny, nz=1, walls_y=True, rho_L=rho, rho_H=rho, tau_L=tau, tau_H=tau,
                   accel=(a, 0.0, 0.0), sigma=1e-4, xi=4.0)
    phi = np.ones((1, ny, 1))
    phi[:, 0, :] = 0.0
    phi[:, -1, :] = 0.0
    o = orc.Oracle(P)
    o.init(phi, np.zeros((3, 1, ny, 1)), np.zeros((1, ny, 1)))
    return o


def test_poiseuille_exact():
    """P11: body-force Poiseuille flow between halfway bounce-back walls at
    y = 1/2 and ny - 3/2.  With the second-order moments at s = 1/(tau+1/2)
    and all odd moments at rate 1, tau = 3/8 makes (1/s - 1/2)(1/1 - 1/2) = 3/16,
    the combination for which halfway bounce-back is exact for a parabola:
    u_x = a/(2 nu) (y - 1/2)(ny - 3/2 - y) must hold to rounding."""
    ny, tau, a = 18, 0.375, 1e-6
    o = _channel(ny, tau, a)
    o.step(20000)
    _, _, _, u = o.state()
    y = np.arange(ny, dtype=float)
    nu = tau / 3.0
    ex = a / (2 * nu) * (y - 0.5) * (ny - 1.5 - y)
    f = slice(1, ny - 1)
    assert np.abs(u[0, 0, f, 0] - ex[f]).max() / ex[f].max() < 1e-9
    assert np.abs(u[1:]).max() < 1e-10 * ex.max()


def test_poiseuille_other_tau():
    """P11 for tau away from 3/8: within 1 % (the halfway bounce-back slip)."""
    ny, a = 18, 1e-6
    for tau in (0.03, 0.3, 1.0):
        o = _channel(ny, tau, a)
        o.step(20000 if tau >= 0.3 else 60000)
        _, _, _, u = o.state()
        y = np.arange(ny, dtype=float)
        ex = a / (2 * tau / 3.0) * (y - 0.5) * (ny - 1.5 - y)
        f = slice(1, ny - 1)
        assert np.abs(u[0, 0, f, 0] - ex[f]).max() / ex[f].max() < 1e-2


def test_layered_poiseuille_viscous_force():
    """Two-layer channel flow (heavy below light, density ratio 10, viscosity
    from the interpolated tau): steady state solves d/dy(mu du/dy) = -rho a with
    mu = rho nu (eq. NSE).  Only the viscous force of eq. viscousForce turns
    the velocity-based scheme's rho d/dy(nu du/dy) into d/dy(rho nu du/dy);
    without it the error here is ~9 %."""
    ny, xi, a, rl, tl, th = 66, 4.0, 1e-6, 0.1, 0.3, 0.375
    yc = (ny - 1) / 2.0
    P = orc.Params(nx=1, ny=ny, nz=1, walls_y=True, rho_L=rl, rho_H=1.0, tau_L=tl, tau_H=th,
                   accel=(a, 0.0, 0.0), sigma=1e-4, xi=xi)
    y = np.arange(ny, dtype=float)
    prof = 0.5 + 0.5 * np.tanh(2 * (yc - y) / xi)
    phi = prof.reshape(1, ny, 1).copy()
    phi[:, 0, :] = 0.0
    phi[:, -1, :] = 0.0
    o = orc.Oracle(P)
    o.init(phi, np.zeros((3, 1, ny, 1)), np.zeros((1, ny, 1)))
    o.step(40000)
    _, _, _, u = o.state()
    yy = np.linspace(0.5, ny - 1.5, 200001)
    f = 0.5 + 0.5 * np.tanh(2 * (yc - yy) / xi)
    rho = rl + f * (1 - rl)
    mu = rho * (tl + f * (th - tl)) / 3.0
    I1 = cumulative_trapezoid(-a * cumulative_trapezoid(rho, yy, initial=0) / mu, yy, initial=0)
    I2 = cumulative_trapezoid(1.0 / mu, yy, initial=0)
    uex = np.interp(y[1:-1], yy, I1 - I1[-1] / I2[-1] * I2)
    err = np.abs(u[0, 0, 1:-1, 0] - uex).max() / np.abs(uex).max()
    assert err < 5e-3, err


def test_hydrostatic_density_jump():
    """Heavy fluid below light fluid at rest under gravity: the pressure
    p = p* rho cs^2 rises by g * integral(rho dy) from top to bottom (1 %) and
    the fluid stays at rest (|u| << g * 1 step).  A wrong sign of the
    pressure force of eq. pressure_force shifts the jump by ~10 %."""
    ny, xi, g, rl = 34, 4.0, 1e-5, 0.1
    yc = (ny - 1) / 2.0
    P = orc.Params(nx=1, ny=ny, nz=1, walls_y=True, rho_L=rl, rho_H=1.0, tau_L=0.3, tau_H=0.3,
                   accel=(0.0, -g, 0.0), sigma=1e-4, xi=xi)
    y = np.arange(ny, dtype=float)
    prof = 0.5 + 0.5 * np.tanh(2 * (yc - y) / xi)
    phi = prof.reshape(1, ny, 1).copy()
    phi[:, 0, :] = 0.0
    phi[:, -1, :] = 0.0
    o = orc.Oracle(P)
    o.init(phi, np.zeros((3, 1, ny, 1)), np.zeros((1, ny, 1)))
    o.step(20000)
    _, _, ph, u = o.state()
    p = o.pressure()[0, :, 0]
    rho = rl + ph[0, :, 0] * (1 - rl)
    jump = p[-2] - p[1]
    expect = -g * (rho[1:-1].sum() - 0.5 * rho[1] - 0.5 * rho[-2])
    assert abs(jump / expect - 1.0) < 1e-2
    assert np.abs(u).max() < 0.1 * g


def test_galilean_advection():
    """A density-matched bubble in a uniform stream U moves with the stream:
    centroid displacement U t within 1 % (tests the velocity terms of the
    phase-field equilibrium phi Gamma(u))."""
    U, steps = 0.02, 300
    s = inputs.Setup(name="adv", nx=48, ny=24, nz=24, walls_y=False, xi=4.0, mobility=0.02,
                     sigma=1e-4, rho_L=1.0, rho_H=1.0, tau_L=0.3, tau_H=0.3, kind="bubble",
                     radius=5.0, center=(12.0, 12.0, 12.0))
    phi, u, ps = inputs.build_fields(s)
    u[0][:] = U
    o = orc.Oracle(_params(s))
    o.init(phi, u, ps)
    c0 = np.array(o.stats()["centroid"])
    o.step(steps)
    c1 = np.array(o.stats()["centroid"])
    assert abs((c1[0] - c0[0]) / (U * steps) - 1.0) < 1e-2
    assert np.abs(c1[1:] - c0[1:]).max() < 1e-2


def test_buoyancy_reference_density_is_a_pressure_gauge():
    """With y walls, F_b = (rho - rho_ref) a for rho_ref = 0 (the printed rho g)
    and for rho_ref = rho_H differ by the uniform force rho_H a, which only
    adds the linear pressure rho_H a.x in the incompressible limit: the bubble
    rises by the same distance.  The printed form also launches the acoustic
    transient of the whole column's weight, which makes its rise velocity
    oscillate around the other one."""
    s = inputs.rising_bubble(12, 40, 12, D=8.0, center=(6.0, 12.0, 6.0), g=2e-5)
    phi, u, ps = inputs.build_fields(s)
    rise = {}
    for ref in (0.0, s.rho_H):
        s.buoyancy_rho_ref = ref
        o = orc.Oracle(_params(s))
        o.init(phi, u, ps)
        y0 = o.stats()["centroid"][1]
        o.step(2000)
        ys = []
        for _ in range(20):          # average over ~8 acoustic periods of the box
            o.step(50)
            ys.append(o.stats()["centroid"][1])
        rise[ref] = np.mean(ys) - y0
    assert rise[s.rho_H] > 0.5
    assert abs(rise[0.0] / rise[s.rho_H] - 1.0) < 0.05


def test_hydrostatic_with_reference_density():
    """rho_ref = rho_H: the heavy fluid feels no body force, the light layer
    on top is pushed up by (rho_L - rho_H) g.  The pressure is flat in the
    heavy bulk and rises with slope (rho_H - rho_L) g in the light bulk
    (1e-3), the jump across the channel is -g * integral(rho - rho_H) dy
    within 3 % (the product-rule discretisation across the 4-cell interface
    is a fixed absolute error, larger here relative to the smaller jump), and
    the fluid stays at rest."""
    ny, xi, g, rl = 34, 4.0, 1e-5, 0.1
    yc = (ny - 1) / 2.0
    P = orc.Params(nx=1, ny=ny, nz=1, walls_y=True, rho_L=rl, rho_H=1.0, tau_L=0.3, tau_H=0.3,
                   accel=(0.0, -g, 0.0), buoyancy_rho_ref=1.0, sigma=1e-4, xi=xi)
    y = np.arange(ny, dtype=float)
    prof = 0.5 + 0.5 * np.tanh(2 * (yc - y) / xi)
    phi = prof.reshape(1, ny, 1).copy()
    phi[:, 0, :] = 0.0
    phi[:, -1, :] = 0.0
    o = orc.Oracle(P)
    o.init(phi, np.zeros((3, 1, ny, 1)), np.zeros((1, ny, 1)))
    o.step(20000)
    _, _, ph, u = o.state()
    p = o.pressure()[0, :, 0]
    rho = rl + ph[0, :, 0] * (1 - rl)
    b = rho - 1.0
    jump = p[-2] - p[1]
    expect = -g * (b[1:-1].sum() - 0.5 * b[1] - 0.5 * b[-2])
    assert abs(jump / expect - 1.0) < 3e-2
    heavy_slope = np.polyfit(y[2:9], p[2:9], 1)[0]
    light_slope = np.polyfit(y[25:32], p[25:32], 1)[0]
    assert abs(heavy_slope) < 1e-3 * g
    assert abs(light_slope / (g * (1.0 - rl)) - 1.0) < 1e-3
    assert np.abs(u).max() < 0.1 * g


def test_density_stays_between_the_phases_in_a_bubble_core():
    """In the core of a small light bubble (rho_H/rho_L = 1000) phi
    oscillates around phi_L by ~1e-3, below phi_L at some steps.  The density
    interpolation is defined between the two phases (eq. density, Sec. 3.2);
    with phi clamped to [phi_L, phi_H] the light fluid keeps rho >= rho_L and
    its velocity grows at most by the buoyant acceleration (1 - rho_L/rho_H)
    g / rho_L ~ 1e-3 per step plus the capillary forcing.  Reading phi
    literally would give rho ~ 1e-6 at phi = -1e-3 and a velocity of ~0.7
    after 6 steps (measured)."""
    s = inputs.rising_bubble(40, 40, 40, D=23.518, center=(20.438, 20.107, 20.264)).with_grid(
        40, 40, 40, walls_y=False)
    phi, u, ps = inputs.build_fields(s)
    o = orc.Oracle(orc.Params(**s.physics()))
    o.init(phi, u, ps)
    phi_min, u_max = 1.0, 0.0
    for _ in range(12):
        o.step(1)
        _, _, ph, uu = o.state()
        phi_min = min(phi_min, float(ph.min()))
        u_max = max(u_max, float(np.sqrt((uu ** 2).sum(0)).max()))
    assert phi_min < -5e-4          # the undershoot happens
    assert u_max < 1e-2             # and does not drive the light fluid


def test_shift_equilibrium_of_an_equilibrium_state_is_the_new_equilibrium():
    """A state at equilibrium has no non-equilibrium part: moving it to new
    fields gives exactly the equilibrium state of those fields (orc_init with
    p* = p / (rho cs^2)), walls untouched."""
    s = inputs.rising_bubble(9, 12, 7, D=5.0, center=(4.0, 5.0, 3.0), g=1e-5).with_grid(9, 12, 7, noise=1e-4)
    P = orc.Params(**s.physics())
    phi0, u0, ps0 = inputs.build_fields(s)
    a = orc.Oracle(P)
    a.init(phi0, u0, ps0)
    rng = np.random.default_rng(5)
    phi1 = phi0 + 0.05 * rng.standard_normal(phi0.shape)
    u1 = u0 + 1e-3 * rng.standard_normal(u0.shape)
    ps1 = 1e-3 * rng.standard_normal(phi0.shape)
    lo, hi = min(s.phi_L, s.phi_H), max(s.phi_L, s.phi_H)
    rho1 = s.rho_L + (np.clip(phi1, lo, hi) - s.phi_L) * (s.rho_H - s.rho_L) / (s.phi_H - s.phi_L)
    a.shift_equilibrium(phi1, u1, ps1 * rho1 / 3.0)
    b = orc.Oracle(P)
    b.init(phi1, u1, ps1)
    fluid = np.ones(phi0.shape, dtype=bool)
    fluid[:, 0, :] = fluid[:, -1, :] = False
    for x, y in zip(a.state(), b.state()):
        if x.ndim == 4:
            x, y = x[:, fluid], y[:, fluid]
        else:
            x, y = x[fluid], y[fluid]
        assert np.abs(x - y).max() <= 1e-15


def test_shift_equilibrium_moments_and_identity():
    """On a developed state: moving to the current fields changes nothing
    (to rounding); moving to new fields gives sum_i G_i = p*' and
    sum_i G_i e_i = j + (u' - u) (the equilibrium moments of Section 3),
    sum_i H_i changes by phi' - phi, and phi_A, u take the new values."""
    s = inputs.rising_bubble(9, 12, 7, D=5.0, center=(4.0, 5.0, 3.0), g=1e-5).with_grid(9, 12, 7, noise=1e-4)
    P = orc.Params(**s.physics())
    o = orc.Oracle(P)
    o.init(*inputs.build_fields(s))
    o.step(6)
    H0, G0, phi0, u0 = o.state()
    p0 = o.pressure()
    o.shift_equilibrium(phi0, u0, p0)
    for x, y in zip(o.state(), (H0, G0, phi0, u0)):
        assert np.abs(x - y).max() <= 1e-16
    rng = np.random.default_rng(6)
    phi1 = phi0 + 0.05 * rng.standard_normal(phi0.shape)
    u1 = u0 + 1e-3 * rng.standard_normal(u0.shape)
    p1 = p0 + 1e-4 * rng.standard_normal(p0.shape)
    o.set_state(H0, G0, phi0, u0)
    o.shift_equilibrium(phi1, u1, p1)
    H1, G1, phi_a, u_a = o.state()
    e27, _ = orc.velocity_set(27)
    fl = np.ones(phi0.shape, dtype=bool)
    fl[:, 0, :] = fl[:, -1, :] = False
    lo, hi = min(s.phi_L, s.phi_H), max(s.phi_L, s.phi_H)
    rho1 = s.rho_L + (np.clip(phi1, lo, hi) - s.phi_L) * (s.rho_H - s.rho_L) / (s.phi_H - s.phi_L)
    assert np.abs(G1.sum(0) - p1 / (rho1 / 3.0))[fl].max() <= 1e-15
    j0 = np.tensordot(e27.T.astype(float), G0, axes=1)
    j1 = np.tensordot(e27.T.astype(float), G1, axes=1)
    assert np.abs(j1 - j0 - (u1 - u0))[:, fl].max() <= 1e-15
    assert np.abs(H1.sum(0) - H0.sum(0) - (phi1 - phi0))[fl].max() <= 1e-15
    assert np.array_equal(phi_a[fl], phi1[fl]) and np.array_equal(u_a[:, fl], u1[:, fl])
    assert np.array_equal(H1[:, ~fl], H0[:, ~fl]) and np.array_equal(G1[:, ~fl], G0[:, ~fl])


def _uniform_stream_bubble(U, rho_L, rho_H, ny=48, center=(11.3, 14.6, 12.2)):
    s = inputs.Setup(name="stream", nx=24, ny=ny, nz=24, walls_y=False, xi=4.0, mobility=0.02,
                     sigma=1e-4, rho_L=rho_L, rho_H=rho_H, tau_L=0.3, tau_H=0.3, kind="bubble",
                     radius=5.0, center=center)
    phi, u, ps = inputs.build_fields(s)
    for a in range(3):
        u[a][:] = U[a]
    return s, phi, u, ps


def test_stats_of_a_uniform_stream():
    """Diagnostics on a state whose answers are fixed without the oracle: a
    light bubble (rho ratio 100) in a uniform stream u = (U_x, U_y, U_z) with
    three different components.  The chi-weighted rise velocity is U_y
    (a weighted mean of a constant); the momentum is U times the total mass of
    fluid, and since rho is linear in phi on [phi_L, phi_H] that total is
    rho_L N + (rho_H - rho_L)/(phi_H - phi_L) (sum phi - phi_L N), with sum phi
    the mass statistic; the largest speed is |U|; the gas volume is
    sum (phi_H - phi)/(phi_H - phi_L) = N - sum phi here."""
    U = (3e-3, -7e-3, 5e-3)
    s, phi, u, ps = _uniform_stream_bubble(U, 0.01, 1.0)
    o = orc.Oracle(_params(s))
    o.init(phi, u, ps)
    st = o.stats()
    N = s.cells
    assert abs(st["mass"] - phi.sum()) <= 1e-12 * phi.sum()
    assert abs(st["gas_volume"] - (N - phi.sum())) <= 1e-12 * N
    assert abs(st["rise_velocity"] - U[1]) <= 16 * EPS64 * abs(U[1])
    mass_of_fluid = s.rho_L * N + (s.rho_H - s.rho_L) * st["mass"]
    for a in range(3):
        assert abs(st["momentum"][a] - U[a] * mass_of_fluid) <= 1e-12 * abs(U[a]) * mass_of_fluid, a
    assert abs(st["max_speed"] - np.sqrt(sum(c * c for c in U))) <= 4 * EPS64


def test_rise_velocity_is_the_gas_weighted_mean():
    """A velocity field linear across the bubble, u_y = U + A (x - x_0): its
    chi-weighted mean is U + A (x_c - x_0) with x_c the chi-weighted centroid
    (both statistics); its plain mean over the box differs (the bubble sits
    off the box centre), so a wrong weighting or a wrong component fails."""
    U, A, x0 = 2e-3, 1e-4, 7.0
    s, phi, u, ps = _uniform_stream_bubble((0.0, U, 0.0), 1.0, 1.0, center=(8.3, 14.6, 12.2))
    xs = np.arange(s.nx, dtype=float)
    u[1] = U + A * (xs[None, None, :] - x0)
    o = orc.Oracle(_params(s))
    o.init(phi, u, ps)
    st = o.stats()
    expect = U + A * (st["centroid"][0] - x0)
    assert abs(st["rise_velocity"] - expect) <= 1e-13 * abs(expect)
    assert abs(u[1].mean() - expect) > 5e-2 * abs(expect)
    # the bubble's centre along y by symmetry of the tanh profile
    assert abs(st["centroid"][1] - 14.6) < 2e-3


def test_bubble_carried_along_y():
    """The y-twin of the Galilean advection pin: a density-matched bubble in
    the uniform stream u = (0, U, 0), periodic in y, moves by U t along y
    within 1 %; its rise velocity stays U within 1 %, and the momentum stays
    U times the fluid mass (rho = 1 everywhere) up to the small net capillary
    force of the discrete interface (1e-4 relative; measured 2e-6)."""
    U, steps = 0.02, 300
    s, phi, u, ps = _uniform_stream_bubble((0.0, U, 0.0), 1.0, 1.0)
    o = orc.Oracle(_params(s))
    o.init(phi, u, ps)
    st0 = o.stats()
    o.step(steps)
    st1 = o.stats()
    c0, c1 = np.array(st0["centroid"]), np.array(st1["centroid"])
    assert abs((c1[1] - c0[1]) / (U * steps) - 1.0) < 1e-2
    assert abs(c1[0] - c0[0]) < 1e-2 and abs(c1[2] - c0[2]) < 1e-2
    assert abs(st1["rise_velocity"] / U - 1.0) < 1e-2
    assert abs(st1["momentum"][1] / (U * s.cells) - 1.0) < 1e-4


def test_init_from_pressure():
    """Equilibrium state of (phi, u, p) (the rebuild after a jump): in the
    heavy bulk the normalised pressure sum_i G_i is p/(rho_H cs^2) = 3 p/rho_H,
    in the light bulk 3 p/rho_L; the pressure read back from the state is p
    everywhere (p = p* rho cs^2, Section 3.2); the velocity moment is u; wall
    rows hold zeros."""
    s = inputs.rising_bubble(10, 14, 9, D=6.0, center=(4.6, 6.3, 4.1), g=1e-5).with_grid(10, 14, 9, noise=1e-4)
    phi, u, _ = inputs.build_fields(s)
    rng = np.random.default_rng(8)
    p = 1e-4 * rng.standard_normal(phi.shape)
    phi[:, 12, :] = s.phi_H                  # a row of each bulk phase
    phi[:, 6, 4] = s.phi_L
    fluid = np.ones(phi.shape, dtype=bool)
    fluid[:, 0, :] = fluid[:, -1, :] = False
    p[~fluid] = 0.0
    o = orc.Oracle(_params(s))
    o.init_pressure(phi, u, p)
    H, G, ph, uu = o.state()
    ps = G.sum(0)
    heavy = fluid & (phi == s.phi_H)
    light = fluid & (phi == s.phi_L)
    assert heavy.any() and light.any()
    # each population is formed as p* w_i + Gamma_i(u) - w_i (the initial-state
    # rule), whose O(w_i) cancellation leaves a rounding of order eps per
    # population: 27 eps bounds the sum
    tol = 27 * EPS64
    assert np.abs(ps[heavy] - 3 * p[heavy] / s.rho_H).max() <= tol
    assert np.abs(ps[light] - 3 * p[light] / s.rho_L).max() <= tol + 4 * EPS64 * np.abs(3 * p / s.rho_L).max()
    assert np.abs(o.pressure() - p)[fluid].max() <= s.rho_H / 3 * tol + 8 * EPS64 * np.abs(p).max()
    e27, _ = orc.velocity_set(27)
    j = np.tensordot(e27.T.astype(float), G, axes=1)
    assert np.abs(j - u)[:, fluid].max() <= tol
    assert np.all(G[:, ~fluid] == 0) and np.all(H[:, ~fluid] == 0)


@pytest.mark.parametrize("literal", [False, True])
def test_density_of_an_overshooting_phase_field(literal):
    """eq. density outside [phi_L, phi_H], read through the equilibrium state of
    a pressure field (p* = p/(rho cs^2)): by default phi is clamped first, so
    phi = 1.5 has rho_H and phi = -0.2 has rho_L; with density_literal the
    printed interpolation rho_L + (phi - phi_L)(rho_H - rho_L)/(phi_H - phi_L)
    holds for every phi (here 1.5 rho_H - 0.5 rho_L and 1.2 rho_L - 0.2 rho_H)."""
    s = inputs.Setup(name="lit", nx=4, ny=3, nz=2, walls_y=False, kind="uniform", rho_L=0.5, rho_H=2.0,
                     tau_L=0.3, tau_H=0.3, xi=4.0, density_literal=literal)
    phi = np.full(s.shape, 0.5)
    phi[0, 0, 0], phi[0, 0, 1] = 1.5, -0.2
    p = np.full(s.shape, 3e-4)
    o = orc.Oracle(_params(s))
    o.init_pressure(phi, np.zeros((3,) + s.shape), p)
    ps = o.state()[1].sum(0)
    rho_over, rho_under = 3e-4 / (ps[0, 0, 0] / 3.0), 3e-4 / (ps[0, 0, 1] / 3.0)
    if literal:
        exp_over, exp_under = 1.5 * s.rho_H - 0.5 * s.rho_L, 1.2 * s.rho_L - 0.2 * s.rho_H
    else:
        exp_over, exp_under = s.rho_H, s.rho_L
    assert abs(rho_over / exp_over - 1.0) < 1e-13
    assert abs(rho_under / exp_under - 1.0) < 1e-13
    assert abs(3e-4 / (ps[0, 1, 0] / 3.0) / (0.5 * (s.rho_L + s.rho_H)) - 1.0) < 1e-13
