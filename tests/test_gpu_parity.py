"""GPU parity: the HIP library (through its C ABI) against the FP64 CPU
oracle on the same seeded inputs.

Bars:
  * FP64 storage: max-abs difference <= 1e-13 after a few steps on small
    ragged grids, <= 1e-11 after 1000 steps of the 32^3 static droplet, on
    every PDF, phi and u.  Both sides evaluate the same formulas in IEEE
    double; the phase-field step follows the oracle's operation order, the
    hydrodynamic collision uses the closed projection form instead of the
    27x27 matrices, so differences are rounding only.
  * FP32 storage, one step from a common state: per quantity
    |gpu - oracle| <= 64 eps32 * scale, scale = max |oracle value| of that
    quantity plus the magnitude of what it is summed from (a sum of 15 or
    27 terms rounded in FP32, then stored in FP32).
  * FP16/BF16 shifted storage, one step from a common state: the rounding
    of the stored shifted value (half an ulp of the format) plus the FP32
    bound.
Full-size checks run the GPU in the same launch configuration as the
benchmark and compare two steps (phase sweep, fused kernel, hydrodynamic
sweep) against the oracle on the whole 128x512x128 grid, and on a sub-box of
the 512^3 grid (cells at least 8 from the sub-box faces, beyond the 6-cell
reach of two coupled steps).
"""
import os
import sys
import time

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2012_06144_amd import inputs

pytestmark = pytest.mark.gpu

EPS32 = float(np.finfo(np.float32).eps)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lbm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2012_06144_amd import lbm as _lbm
    return _lbm


def _pair(lbm, setup, storage="f64"):
    phi, u, ps = inputs.build_fields(setup)
    o = orc.Oracle(orc.Params(**setup.physics()))
    o.init(phi, u, ps)
    g = lbm.Solver(setup.physics(), storage=storage)
    g.init_fields(phi, u, ps)
    return o, g


def _maxdiff(a, b):
    return [float(np.abs(x - y).max()) for x, y in zip(a, b)]


SMALL = {
    "ragged_walls_bubble": lambda: inputs.rising_bubble(13, 21, 9, D=8.0, center=(6.0, 9.0, 4.0), g=1e-5)
    .with_grid(13, 21, 9, noise=1e-4),
    "periodic_droplet": lambda: inputs.static_droplet(n=16, R=5.0, noise=1e-5),
    "channel_1x18x1": lambda: inputs.Setup(name="ch", nx=1, ny=18, nz=1, walls_y=True, kind="uniform",
                                           rho_L=1.0, rho_H=1.0, tau_L=0.375, tau_H=0.375,
                                           accel=(1e-5, 0.0, 0.0), xi=4.0, sigma=1e-4),
    "one_fluid_row": lambda: inputs.rising_bubble(12, 3, 10, D=4.0, center=(6.0, 1.0, 5.0), g=1e-5)
    .with_grid(12, 3, 10, noise=1e-4),
    "bubble_core_undershoot": lambda: inputs.rising_bubble(40, 40, 40, D=23.518, center=(20.438, 20.107, 20.264))
    .with_grid(40, 40, 40, walls_y=False),
    "cube_2": lambda: inputs.static_droplet(n=2, R=0.7, noise=1e-3),
    "cube_1": lambda: inputs.Setup(name="c1", nx=1, ny=1, nz=1, walls_y=False, kind="uniform",
                                   noise=1e-3, rho_L=1.0, rho_H=10.0, tau_L=1.0, tau_H=1.0, xi=4.0),
}


@pytest.mark.parametrize("case", list(SMALL))
def test_init_matches_oracle_f64(lbm, case):
    _say(f"[gpu] init parity {case}")
    o, g = _pair(lbm, SMALL[case]())
    d = _maxdiff(o.state(), g.state())
    assert max(d) <= 1e-15, d


@pytest.mark.parametrize("case", list(SMALL))
@pytest.mark.parametrize("steps", [1, 7])
@pytest.mark.parametrize("zmarch", ["0", "1"])
def test_steps_match_oracle_f64(lbm, case, steps, zmarch, monkeypatch):
    """FP64 steps against the oracle on the default sweeps (one cell per
    thread, the fused kernel for steps >= 2) and on the z-marching sweeps that
    stage the phase field of three planes in LDS (LBM_ZMARCH=1)."""
    monkeypatch.setenv("LBM_ZMARCH", zmarch)
    _say(f"[gpu] step parity {case} steps={steps} zmarch={zmarch}")
    o, g = _pair(lbm, SMALL[case]())
    o.step(steps)
    g.step(steps)
    d = _maxdiff(o.state(), g.state())
    assert max(d) <= 1e-13, d


def test_literal_density_matches_oracle_f64(lbm):
    """density_literal = 1 (eq. density and the tau interpolation for every
    phi, no clamp) on the 16^3 droplet, whose phase field leaves [0, 1]
    slightly within 7 steps: GPU and oracle agree to 1e-13, and the literal
    run differs from the default clamped run (the switch takes effect)."""
    s = SMALL["periodic_droplet"]().with_grid(16, 16, 16, density_literal=True)
    o, g = _pair(lbm, s)
    o.step(7)
    g.step(7)
    lit = g.state()
    d = _maxdiff(o.state(), lit)
    _say(f"[gpu] literal density 7 steps: {d}")
    assert max(d) <= 1e-13, d
    _, gc = _pair(lbm, SMALL["periodic_droplet"]())
    gc.step(7)
    assert max(_maxdiff(gc.state(), lit)) > 1e-12


def test_static_droplet_1000_steps_f64(lbm):
    """32^3 static droplet, R = 8, xi = 4, rho 10/1, sigma 1e-3, seeded
    velocity noise: after 1000 steps every PDF, phi and u within 1e-11."""
    s = inputs.static_droplet()
    _say(f"[gpu] static droplet 1000 steps {s.shape}")
    o, g = _pair(lbm, s)
    m0 = g.reduce_mass()
    t = time.time()
    o.step(s.steps)
    _say(f"  oracle {time.time() - t:.1f}s")
    g.step(s.steps)
    d = _maxdiff(o.state(), g.state())
    _say(f"  max|dH|,|dG|,|dphi|,|du| = {d}")
    assert max(d) <= 1e-11, d
    m1 = g.reduce_mass()
    assert abs(m1 - m0) / m0 <= 4 * np.finfo(np.float64).eps * s.steps
    _check_stats(s, o, g, d)
    _check_pressure(s, o, g, d)


EPS64 = float(np.finfo(np.float64).eps)


def _check_stats(s, o, g, d):
    """Every statistic of lbm_reduce_stats against the oracle's, within what
    the field differences d = (dH, dG, dphi, du) allow plus FP64 rounding of
    the sums (they are summed in different orders): with dchi = dphi/(phi_H -
    phi_L), N fluid cells and L the largest coordinate,
      sums of phi-functions:  |d| <= 8 N dchi + 64 N eps |value|/N,
      centroid:               |d| <= 2 N L dchi / V_g + rounding,
      rise velocity:          |d| <= du + 2 N dchi (u_max + |U|) / V_g + rounding,
      momentum:               |d| <= N (rho_H du + drho dchi u_max) + rounding,
      max speed:              |d| <= sqrt(3) du + rounding."""
    so, sg = o.stats(), g.stats()
    _, _, dphi, du = d
    N = s.nx * s.nz * (s.ny - 2 if s.walls_y else s.ny)
    dchi = dphi / abs(s.phi_H - s.phi_L)
    L = max(s.nx, s.ny, s.nz)
    rnd = 64 * N * EPS64
    umax = so["max_speed"]
    Vg = so["gas_volume"]
    _say(f"  stats oracle {so}")
    for k in ("mass", "gas_volume", "interface_sum", "grad_sum"):
        assert abs(sg[k] - so[k]) <= 8 * N * dchi + rnd * abs(so[k]) / N + 1e-300, (k, sg[k], so[k])
    rel = lambda k: (8 * N * dchi + rnd * abs(so[k]) / N) / abs(so[k])
    assert abs(sg["xi_eff"] - so["xi_eff"]) <= (rel("interface_sum") + rel("grad_sum")) * so["xi_eff"]
    cb = 2 * N * L * dchi / Vg + 2 * rnd * L / N
    assert np.abs(np.array(sg["centroid"]) - np.array(so["centroid"])).max() <= cb, (sg["centroid"], so["centroid"])
    U = so["rise_velocity"]
    ub = du + 2 * N * dchi * (umax + abs(U)) / Vg + 2 * rnd * (umax + abs(U)) / N
    assert abs(sg["rise_velocity"] - U) <= ub, (sg["rise_velocity"], U, ub)
    rho_max = max(s.rho_L, s.rho_H)
    mb = N * (rho_max * du + abs(s.rho_H - s.rho_L) * dchi * umax) + rnd * rho_max * umax
    assert np.abs(np.array(sg["momentum"]) - np.array(so["momentum"])).max() <= mb, (sg["momentum"], so["momentum"])
    assert abs(sg["max_speed"] - umax) <= np.sqrt(3.0) * du + 4 * EPS64 * umax


def _check_pressure(s, o, g, d):
    """Pressure p = p* rho c_s^2 of lbm_get_macroscopic against orc_pressure:
    with p* = sum_i G_i (27 terms) and rho linear in phi,
    |dp| <= c_s^2 (rho_max 27 (dG + eps max|G|) + max|p*| drho dchi) + 4 eps |p|."""
    po, pg = o.pressure(), g.pressure()
    _, G, _, _ = o.state()
    dG, dphi = d[1], d[2]
    ps = np.abs(G.sum(0)).max()
    rho_max = max(s.rho_L, s.rho_H)
    bound = (rho_max * 27 * (dG + EPS64 * np.abs(G).max()) + ps * abs(s.rho_H - s.rho_L) * dphi
             / abs(s.phi_H - s.phi_L)) / 3.0 + 4 * EPS64 * np.abs(po).max()
    err = float(np.abs(pg - po).max())
    _say(f"  max|dp| = {err:.3e} (bound {bound:.3e}, max|p| {np.abs(po).max():.3e})")
    assert err <= bound


LONG_WALL = {
    # 13 x 21 x 9 with walls, a D = 8 bubble under gravity, rising-bubble
    # physics (rho 1 / 0.001, tau 0.03 / 0.3, xi 5, sigma 1e-4, M 0.02)
    "ragged_walls_bubble": SMALL["ragged_walls_bubble"],
    # the rising-bubble workload at reduced width: 24 x 64 x 24, D = 12 at an
    # off-node centre, Eo = g rho_H D^2 / sigma = 10
    "rising_bubble_24x64x24": lambda: inputs.rising_bubble(24, 64, 24, D=12.0, center=(11.7, 18.3, 12.2),
                                                           g=10 * 1e-4 / 144.0).with_grid(24, 64, 24, noise=1e-5),
}


@pytest.mark.parametrize("case", list(LONG_WALL))
def test_walls_gravity_1000_steps_f64(lbm, case):
    """The rising-bubble physics (walls, gravity, density ratio 1000) over
    1000 FP64 steps on the default path (one phase sweep, 999 fused kernels,
    one hydrodynamic sweep): every PDF, phi and u within 1e-11 of the oracle;
    the pressure, the rise velocity, the centroid and every other statistic
    within the bounds the field differences allow; sum(phi) conserved."""
    s = LONG_WALL[case]()
    _say(f"[gpu] walls+gravity 1000 steps {case} {s.shape}")
    o, g = _pair(lbm, s)
    m0 = g.reduce_mass()
    t = time.time()
    o.step(1000)
    _say(f"  oracle {time.time() - t:.1f}s")
    g.step(1000)
    d = _maxdiff(o.state(), g.state())
    _say(f"  max|dH|,|dG|,|dphi|,|du| = {d}")
    assert max(d) <= 1e-11, d
    m1 = g.reduce_mass()
    assert abs(m1 - m0) / m0 <= 4 * EPS64 * 1000
    so = o.stats()
    assert so["rise_velocity"] > 0 and so["max_speed"] > 1e-4     # the bubble does rise
    _check_stats(s, o, g, d)
    _check_pressure(s, o, g, d)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_set_macroscopic_matches_oracle(lbm, storage):
    """lbm_set_macroscopic (the rebuild at equilibrium after a jump) from
    (phi, u, p) against the oracle's equilibrium state of the same fields with
    p* = p/(rho c_s^2): FP64 within a few eps per population (the equilibrium
    is summed in a different order), FP32 within the FP32 step bound; the
    pressure read back agrees too."""
    import torch
    s = SMALL["ragged_walls_bubble"]()
    o, _ = _pair(lbm, s)
    o.step(5)
    _, _, phi, u = o.state()
    rng = np.random.default_rng(29)
    p = o.pressure() + 1e-5 * rng.standard_normal(phi.shape)
    dt = torch.float64 if storage == "f64" else torch.float32
    if dt == torch.float32:
        phi, u, p = (a.astype(np.float32).astype(np.float64) for a in (phi, u, p))
    ref = orc.Oracle(orc.Params(**s.physics()))
    ref.init_pressure(phi, u, p)
    g = lbm.Solver(s.physics(), storage=storage)
    g.set_macroscopic(*(torch.from_numpy(a).to(dt).cuda() for a in (phi, u, p)))
    rst, gst = ref.state(), g.state()
    d = _maxdiff(rst, gst)
    _say(f"[gpu] set_macroscopic {storage}: {d}")
    if storage == "f64":
        tol = [32 * EPS64 * max(1.0, np.abs(x).max()) for x in rst]
    else:
        tol = [64 * EPS32 * max(1.0, np.abs(x).max()) for x in rst]
    assert all(x <= t for x, t in zip(d, tol)), (d, tol)
    fluid = np.ones(s.shape, dtype=bool)
    fluid[:, 0, :] = fluid[:, -1, :] = False
    dp = np.abs(g.pressure() - ref.pressure())[fluid].max()
    scale = max(s.rho_L, s.rho_H) / 3.0 * 27 * tol[1] + 4 * (EPS64 if storage == "f64" else EPS32) * np.abs(p).max()
    assert dp <= scale, (dp, scale)


def test_set_get_roundtrip(lbm):
    s = SMALL["ragged_walls_bubble"]()
    o, g = _pair(lbm, s)
    o.step(3)
    st = o.state()
    g.set_state(*st)
    assert max(_maxdiff(st, g.state())) == 0.0
    f32 = lbm.Solver(s.physics(), storage="f32")
    f32.set_state(*st)
    back = f32.state()
    for a, b in zip(st, back):
        assert np.array_equal(b, a.astype(np.float32).astype(np.float64))


def _fp32_tolerances(ost, src):
    """64 eps32 times the scale of each output.  The phase-field rest
    population is formed as phi minus the 14 others, so H and phi scale with
    the 15-term sum; G and u scale with the 27 hydrodynamic PDFs they are
    summed from."""
    H0, G0, phi0, u0 = src
    sphi = max(15 * np.abs(H0).max(), np.abs(ost[2]).max())
    sH = max(np.abs(H0).max(), np.abs(ost[0]).max(), sphi)
    sG = max(27 * np.abs(G0).max(), np.abs(ost[1]).max())  # g_eq has no O(w) cancellation
    su = max(27 * np.abs(G0).max(), np.abs(ost[3]).max())
    return [64 * EPS32 * v for v in (sH, sG, sphi, su)]


def test_one_step_f32_small(lbm):
    s = SMALL["ragged_walls_bubble"]()
    o, g = _pair(lbm, s, storage="f32")
    g.step(5)
    src = g.state()
    o.set_state(*src)
    o.step(1)
    g.step(1)
    ost = o.state()
    d = _maxdiff(ost, g.state())
    tol = _fp32_tolerances(ost, src)
    _say(f"[gpu] f32 one step diffs {d} tol {tol}")
    assert all(x <= t for x, t in zip(d, tol)), (d, tol)


def _ulp(v, fmt):
    """Spacing of the stored format at |v| in unscaled units: FP16 values are
    stored times 2^10, which moves the subnormal range down by 2^10."""
    mant, emin = (10, -24) if fmt == "f16s" else (7, -126)
    e = np.floor(np.log2(np.maximum(np.abs(v), 2.0 ** emin)))
    return 2.0 ** (e - mant)


def _w(q):
    return orc.velocity_set(q)[1].reshape(q, 1, 1, 1)


def _lowp_bounds(ost, gst, tol, fmt):
    """Per-population bounds for 16-bit storage of h_i - phi w_i and g_i / w_i:
    half an ulp of the stored value (in stored units), the FP32 bound and
    the FP32 rounding of the decode."""
    shift = gst[2][None] * _w(15)            # the GPU's new phi times w_i
    bound_H = 0.5 * _ulp(ost[0] - shift, fmt) + tol[0] + EPS32 * (np.abs(ost[0]) + np.abs(shift))
    bound_G = 0.5 * _ulp(ost[1] / _w(27), fmt) * _w(27) + tol[1] + EPS32 * np.abs(ost[1])
    return bound_H, bound_G


LOWP_GRIDS = {
    # odd nz: one-cell-per-thread sweeps on the paired storage layout
    "ragged_walls_bubble": SMALL["ragged_walls_bubble"],
    # even nz: paired sweeps (cells z and z + nz/2 in one 32-bit word)
    "walls_bubble_even_nz": lambda: inputs.rising_bubble(13, 21, 10, D=8.0, center=(6.0, 9.0, 4.0), g=1e-5)
    .with_grid(13, 21, 10, noise=1e-4),
    "periodic_droplet": SMALL["periodic_droplet"],
}


@pytest.mark.parametrize("grid", list(LOWP_GRIDS))
@pytest.mark.parametrize("fmt", ["f16s", "bf16s"])
def test_one_step_low_precision_small(lbm, fmt, grid):
    """16-bit storage of h_i - phi w_i and g_i / w_i: one step from a common
    state is within half an ulp of the stored value (in stored units) plus the
    FP32 bound plus the FP32 rounding of the decode."""
    s = LOWP_GRIDS[grid]()
    o, g = _pair(lbm, s, storage=fmt)
    g.step(5)
    src = g.state()
    o.set_state(*src)
    o.step(1)
    g.step(1)
    ost, gst = o.state(), g.state()
    tol = _fp32_tolerances(ost, src)
    bound_H, bound_G = _lowp_bounds(ost, gst, tol, fmt)
    # the rest population closes sum(h) = phi on the decoded values of the
    # other 14, so it carries their rounding too
    bound_H[0] += 0.5 * _ulp(ost[0][1:] - gst[2][None] * _w(15)[1:], fmt).sum(axis=0) + 15 * EPS32 * np.abs(gst[2])
    fluid = np.ones(s.shape, dtype=bool)
    if s.walls_y:
        fluid[:, 0, :] = fluid[:, -1, :] = False
    dH = np.abs(gst[0] - ost[0])[:, fluid]
    dG = np.abs(gst[1] - ost[1])[:, fluid]
    _say(f"[gpu] {fmt}: max dH/bound {np.max(dH / bound_H[:, fluid]):.3f} "
         f"max dG/bound {np.max(dG / bound_G[:, fluid]):.3f}")
    assert np.all(dH <= bound_H[:, fluid])
    assert np.all(dG <= bound_G[:, fluid])
    # phi and u are summed from the common decoded inputs in FP32 and kept in FP32
    assert np.abs(gst[2] - ost[2]).max() <= tol[2]
    assert np.abs(gst[3] - ost[3]).max() <= tol[3]


@pytest.mark.parametrize("grid", ["walls_bubble_even_nz", "periodic_droplet"])
@pytest.mark.parametrize("fmt", ["f16s", "bf16s"])
def test_paired_sweeps_match_per_cell_sweeps(lbm, fmt, grid, monkeypatch):
    """The paired 16-bit sweeps (one thread per cells z, z + nz/2, 32-bit
    words) compute exactly what the one-cell-per-thread sweeps compute on the
    same storage: 7 steps, every stored population, phi and u identical."""
    s = LOWP_GRIDS[grid]()
    assert s.nz % 2 == 0
    phi, u, ps = inputs.build_fields(s)
    states = []
    for pair in ("0", "1"):
        monkeypatch.setenv("LBM_PAIR", pair)
        g = lbm.Solver(s.physics(), storage=fmt)
        g.init_fields(phi, u, ps)
        g.step(7)
        states.append(g.state())
    for a, b in zip(*states):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("storage", ["f64", "f32", "f16s", "bf16s"])
@pytest.mark.parametrize("case", ["ragged_walls_bubble", "walls_bubble_even_nz", "periodic_droplet"])
def test_shift_equilibrium_matches_oracle(lbm, storage, case):
    """Moving a developed state to perturbed macroscopic fields with the
    non-equilibrium parts kept (lbm_shift_equilibrium) against the oracle
    applied to the GPU's own canonical state: FP64 to rounding, FP32 within
    the FP32 bounds of the sweeps, 16-bit within half an ulp of the stored
    format on top."""
    import torch
    s = (LOWP_GRIDS[case] if case in LOWP_GRIDS else SMALL[case])()
    _say(f"[gpu] shift_equilibrium {storage} {case} {s.shape}")
    o, g = _pair(lbm, s, storage=storage)
    g.step(5)
    src = g.state()
    o.set_state(*src)
    rng = np.random.default_rng(41)
    phi1 = src[2] + 0.02 * rng.standard_normal(s.shape)
    u1 = src[3] + 1e-3 * rng.standard_normal((3,) + s.shape)
    p1 = o.pressure() + 1e-4 * rng.standard_normal(s.shape)
    o.shift_equilibrium(phi1, u1, p1)
    ost = o.state()
    dt = torch.float64 if storage == "f64" else torch.float32
    if dt == torch.float32:                  # the oracle sees the fields the GPU is given
        phi1, u1, p1 = (a.astype(np.float32).astype(np.float64) for a in (phi1, u1, p1))
        o.set_state(*src)
        o.shift_equilibrium(phi1, u1, p1)
        ost = o.state()
    g.set_macroscopic(*(torch.from_numpy(a).to(dt).cuda() for a in (phi1, u1, p1)), keep_neq=True)
    gst = g.state()
    d = _maxdiff(ost, gst)
    _say(f"  max|dH|,|dG|,|dphi|,|du| = {d}")
    if storage == "f64":
        assert max(d) <= 1e-14, d
        return
    tol = _fp32_tolerances(ost, src)
    if storage == "f32":
        assert all(x <= t for x, t in zip(d, tol)), (d, tol)
        return
    # the source state holds the decoded stored values, so the move rounds once
    bound_H, bound_G = _lowp_bounds(ost, gst, tol, storage)
    assert np.all(np.abs(gst[0] - ost[0]) <= bound_H)
    assert np.all(np.abs(gst[1] - ost[1]) <= bound_G)
    assert d[2] <= tol[2] and d[3] <= tol[3]


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("case", ["ragged_walls_bubble", "periodic_droplet"])
def test_fused_steps_match_separate_sweeps(lbm, storage, case, monkeypatch):
    """lbm_step with the hydrodynamic sweep of each step fused to the phase
    sweep of the next (LBM_FUSE=1) gives bit-identical states to the
    separate sweeps for n = 1, 2 and 5 steps; FP64 also against the oracle."""
    s = SMALL[case]()
    phi, u, ps = inputs.build_fields(s)
    _say(f"[gpu] fused steps {storage} {case}")
    for nsteps in (1, 2, 5):
        states = {}
        for fuse in ("0", "1"):
            monkeypatch.setenv("LBM_FUSE", fuse)
            g = lbm.Solver(s.physics(), storage=storage)
            g.init_fields(phi, u, ps)
            g.step(nsteps)
            g.step(1)
            states[fuse] = g.state()
            del g
        for a, b in zip(states["0"], states["1"]):
            assert np.array_equal(a, b), nsteps
    if storage == "f64":
        o = orc.Oracle(orc.Params(**s.physics()))
        o.init(phi, u, ps)
        o.step(6)
        assert max(_maxdiff(o.state(), states["1"])) <= 1e-13


def test_step_timed_fused(lbm, monkeypatch):
    """The timed fused steps return a positive mean kernel time and leave the
    state lbm_step leaves; 16-bit storage has no fused kernel (LBM_EARG)."""
    s = SMALL["ragged_walls_bubble"]()
    phi, u, ps = inputs.build_fields(s)
    monkeypatch.setenv("LBM_PAIR", "0")
    st = {}
    for timed in (False, True):
        g = lbm.Solver(s.physics(), storage="f32")
        g.init_fields(phi, u, ps)
        if timed:
            ms = g.step_timed_fused(4)
            assert ms > 0.0
        else:
            g.step(4)
        st[timed] = g.state()
        del g
    for a, b in zip(st[False], st[True]):
        assert np.array_equal(a, b)
    g = lbm.Solver(s.physics(), storage="f16s")
    g.init_fields(phi, u, ps)
    with pytest.raises(lbm.LbmError):
        g.step_timed_fused(4)
    with pytest.raises(lbm.LbmError):
        g.step_timed_fused(1)


def test_stream_copy(lbm):
    import torch
    a = torch.randint(0, 2 ** 31, (1 << 20,), dtype=torch.int32, device="cuda")
    b = torch.zeros_like(a)
    lbm.lbm_stream_copy(a, b, a.numel() * 4, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_step_argument_errors(lbm):
    s = SMALL["periodic_droplet"]()
    _, g = _pair(lbm, s)
    with pytest.raises(lbm.LbmError, match="n must be"):
        g.step(0)
    with pytest.raises(lbm.LbmError):
        lbm.lbm_get_macroscopic(g.ctx, 5, None, None, None)


def test_rising_bubble_full_grid_two_steps_f64(lbm):
    """Full 128x512x128 rising-bubble grid (walls, gravity), FP64: 30 GPU
    steps, then two steps on both sides from the GPU's state, all cells; the
    GPU's two steps run the phase sweep, one fused kernel (hydrodynamic sweep
    of the first step with the phase sweep of the second) and the
    hydrodynamic sweep, as every multi-step lbm_step does."""
    s = inputs.rising_bubble()
    _say(f"[gpu] full-grid one-step parity {s.shape} f64")
    phi, u, ps = inputs.build_fields(s)
    g = lbm.Solver(s.physics(), storage="f64")
    g.init_fields(phi, u, ps)
    g.step(30)
    src = g.state()
    o = orc.Oracle(orc.Params(**s.physics()))
    o.set_state(*src)
    del src
    t = time.time()
    o.step(2)
    _say(f"  oracle 2 steps {time.time() - t:.1f}s")
    g.step(2)
    d = _maxdiff(o.state(), g.state())
    _say(f"  diffs {d}")
    assert max(d) <= 1e-13, d


def test_bubble_swarm_512_subbox_two_steps_f32(lbm):
    """512^3 bubble swarm in FP32 storage (the benchmark workload and launch
    configuration, so the two steps run the fused kernel the benchmark
    times): 20 steps, then two steps compared with the oracle on a
    64 x 512 x 64 sub-box around a bubble, on cells at least 8 from the
    sub-box faces (one coupled step reaches 3 cells).  The first step's FP32
    rounding is carried into the second, so the one-step bound doubles."""
    import torch
    s = inputs.bubble_swarm()
    _say(f"[gpu] 512^3 sub-box parity f32")
    phi, u, ps = inputs.build_fields(s)
    g = lbm.Solver(s.physics(), storage="f32")
    g.init_fields(phi, u, ps)
    del phi, u, ps
    m0 = g.reduce_mass()
    g.step(20)
    cx, cy, cz = s.extra["centres"][0]
    W, M = 64, 8
    x0 = int(cx) - W // 2
    z0 = int(cz) - W // 2
    xs = torch.arange(x0, x0 + W, device="cuda") % s.nx
    zs = torch.arange(z0, z0 + W, device="cuda") % s.nz

    def sub():
        H, G = g.pdfs()
        phi, uu, _ = g.macroscopic(torch.float64)
        out = []
        for t in (H, G, phi, uu):
            t = t.index_select(-1, xs).index_select(-3, zs)
            out.append(t.cpu().numpy())
        del H, G, phi, uu
        torch.cuda.empty_cache()
        return out

    src = sub()
    phys = s.physics()
    phys.update(nx=W, nz=W)
    o = orc.Oracle(orc.Params(**phys))
    o.set_state(*src)
    o.step(2)
    g.step(2)
    ost, gst = o.state(), sub()
    tol = [2 * t for t in _fp32_tolerances(ost, src)]
    inner = (slice(None), slice(M, W - M), slice(None), slice(M, W - M))
    d = [float(np.abs(a[inner] - b[inner]).max()) if a.ndim == 4 else
         float(np.abs(a[inner[1:]] - b[inner[1:]]).max()) for a, b in zip(ost, gst)]
    _say(f"  diffs {d} tol {tol}")
    assert all(x <= t for x, t in zip(d, tol)), (d, tol)
    m1 = g.reduce_mass()
    _say(f"  mass drift over 22 steps (f32 storage): {(m1 - m0) / m0:.3e}")
    assert abs(m1 - m0) / m0 < 1e-6
