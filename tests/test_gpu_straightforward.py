"""GPU parity of the straightforward algorithm (lbm_step_straightforward:
six kernels per step, Alg. naiveAlgorithm of Sec. 4.2, time-consistent
reading) against the oracle's straightforward step, through the C ABI.

Bars as for the improved step: FP64 within 1e-13 after 1 and 7 steps on
small ragged grids and within 1e-11 after 1000 steps of the rising-bubble
physics on a small grid with walls; FP32 one step from a common state within
64 eps32 times the scale of each quantity.  The improved and straightforward
steps can be mixed on one context (same stored state).
"""
import sys
import time

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2012_06144_amd import inputs

pytestmark = pytest.mark.gpu

EPS32 = float(np.finfo(np.float32).eps)
EPS64 = float(np.finfo(np.float64).eps)


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


CASES = {
    "ragged_walls_bubble": lambda: inputs.rising_bubble(13, 21, 9, D=8.0, center=(6.0, 9.0, 4.0), g=1e-5)
    .with_grid(13, 21, 9, noise=1e-4),
    "periodic_droplet": lambda: inputs.static_droplet(n=16, R=5.0, noise=1e-5),
    "channel_1x18x1": lambda: inputs.Setup(name="ch", nx=1, ny=18, nz=1, walls_y=True, kind="uniform",
                                           rho_L=1.0, rho_H=1.0, tau_L=0.375, tau_H=0.375,
                                           accel=(1e-5, 0.0, 0.0), xi=4.0, sigma=1e-4),
    "one_fluid_row": lambda: inputs.rising_bubble(12, 3, 10, D=4.0, center=(6.0, 1.0, 5.0), g=1e-5)
    .with_grid(12, 3, 10, noise=1e-4),
    "cube_2": lambda: inputs.static_droplet(n=2, R=0.7, noise=1e-3),
    # more than one block of cells, ragged tail
    "bubble_33x40x17": lambda: inputs.rising_bubble(33, 40, 17, D=12.0, center=(16.2, 15.1, 8.3), g=1e-5)
    .with_grid(33, 40, 17, noise=1e-5),
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("steps", [1, 7])
def test_straightforward_matches_oracle_f64(lbm, case, steps):
    _say(f"[gpu] straightforward parity {case} steps={steps}")
    o, g = _pair(lbm, CASES[case]())
    o.step_straightforward(steps)
    g.step_straightforward(steps)
    d = _maxdiff(o.state(), g.state())
    assert max(d) <= 1e-13, d


def test_straightforward_1000_steps_walls_gravity_f64(lbm):
    """The rising-bubble physics (walls, gravity, density ratio 1000) over
    1000 straightforward FP64 steps: every PDF, phi and u within 1e-11 of the
    oracle, sum(phi) conserved, the rise velocity within the field bound."""
    s = CASES["ragged_walls_bubble"]()
    _say(f"[gpu] straightforward 1000 steps {s.shape}")
    o, g = _pair(lbm, s)
    m0 = g.reduce_mass()
    t = time.time()
    o.step_straightforward(1000)
    _say(f"  oracle {time.time() - t:.1f}s")
    g.step_straightforward(1000)
    d = _maxdiff(o.state(), g.state())
    _say(f"  max|dH|,|dG|,|dphi|,|du| = {d}")
    assert max(d) <= 1e-11, d
    assert abs(g.reduce_mass() - m0) / m0 <= 4 * EPS64 * 1000
    so, sg = o.stats(), g.stats()
    assert so["rise_velocity"] > 0
    assert abs(so["rise_velocity"] - sg["rise_velocity"]) <= 1e-9 * max(1.0, abs(so["rise_velocity"]))


def test_mixed_algorithms_f64(lbm):
    """The two algorithms leave the same kind of state: 3 improved, 4
    straightforward and 3 improved steps match the oracle doing the same."""
    s = CASES["ragged_walls_bubble"]()
    o, g = _pair(lbm, s)
    for k, fn in ((3, "step"), (4, "step_straightforward"), (3, "step")):
        getattr(o, fn)(k)
        getattr(g, fn)(k)
    d = _maxdiff(o.state(), g.state())
    assert max(d) <= 1e-13, d


def test_straightforward_one_step_f32(lbm):
    """FP32 storage, one straightforward step from a common state: 64 eps32
    times the scale of each quantity (as for the improved step)."""
    s = CASES["bubble_33x40x17"]()
    o, g = _pair(lbm, s, storage="f32")
    g.step_straightforward(5)
    src = g.state()
    o.set_state(*src)
    o.step_straightforward(1)
    g.step_straightforward(1)
    ost = o.state()
    H0, G0, phi0, u0 = src
    sphi = max(15 * np.abs(H0).max(), np.abs(ost[2]).max())
    scales = [max(np.abs(H0).max(), np.abs(ost[0]).max(), sphi), max(27 * np.abs(G0).max(), np.abs(ost[1]).max()),
              sphi, max(27 * np.abs(G0).max(), np.abs(ost[3]).max())]
    tol = [64 * EPS32 * v for v in scales]
    d = _maxdiff(ost, g.state())
    _say(f"[gpu] straightforward f32 one step diffs {d} tol {tol}")
    assert all(x <= t for x, t in zip(d, tol)), (d, tol)


@pytest.mark.parametrize("storage", ["f16s", "bf16s"])
def test_straightforward_rejects_16bit_storage(lbm, storage):
    s = CASES["periodic_droplet"]()
    g = lbm.Solver(s.physics(), storage=storage)
    g.init_fields(*inputs.build_fields(s))
    with pytest.raises(lbm.LbmError, match="FP64 or FP32"):
        g.step_straightforward(1)
