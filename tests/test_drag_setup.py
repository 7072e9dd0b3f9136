"""Host checks of the drag-coefficient study (Sec. 6.1): the workload builder
reproduces the dimensionless groups it is given, and the two drag formulas
have their closed-form limits."""
import math

import pytest

from paper_2012_06144_amd import inputs, studies


@pytest.mark.parametrize("re", [10.0, 30.0, 120.0])
def test_drag_bubble_has_the_requested_groups(re):
    s = inputs.drag_bubble(re, eo=30.0, D=32.0, t_ref=2000.0)
    g = -s.accel[1]
    D = 2 * s.radius
    mu_H = s.rho_H * s.tau_H / 3.0          # nu = tau cs^2
    mu_L = s.rho_L * s.tau_L / 3.0
    assert math.isclose(s.rho_H * math.sqrt(g * D ** 3) / mu_H, re, rel_tol=1e-12)
    assert math.isclose(g * s.rho_H * D * D / s.sigma, 30.0, rel_tol=1e-12)
    assert math.isclose(math.sqrt(D / g), 2000.0, rel_tol=1e-12)
    assert math.isclose(s.rho_H / s.rho_L, 1000.0, rel_tol=1e-12)
    assert math.isclose(mu_H / mu_L, 100.0, rel_tol=1e-12)
    assert (s.nx, s.ny, s.nz) == (256, 1024, 256) and s.walls_y
    assert s.center == (128.0, 256.0, 128.0) and s.xi == 5.0 and s.mobility == 0.04


def test_bhaga_weber_limits():
    # Re -> infinity leaves the constant 2.67; at Re = 16 both terms are 2.67^0.9 and 1
    assert math.isclose(studies.drag_coefficient_bhaga_weber(1e12), 2.67, rel_tol=1e-9)
    assert math.isclose(studies.drag_coefficient_bhaga_weber(16.0), (2.67 ** 0.9 + 1.0) ** (10.0 / 9.0),
                        rel_tol=1e-15)
    # low Re: Stokes-like 16/Re
    assert math.isclose(studies.drag_coefficient_bhaga_weber(1e-6), 16.0 / 1e-6, rel_tol=1e-4)


def test_drag_from_terminal_velocity():
    # C_D = 4/3 g (rho_H - rho_L) D / (rho_H u_t^2): a bubble whose drag balances its buoyancy
    g, D, rh, rl, u = 8e-6, 32.0, 1.0, 1e-3, 5e-3
    cd = studies.drag_coefficient_lbm(g, rh, rl, D, u)
    assert math.isclose(cd * rh * u * u * (math.pi * D * D / 4) / 2,
                        (rh - rl) * g * math.pi * D ** 3 / 6, rel_tol=1e-12)
