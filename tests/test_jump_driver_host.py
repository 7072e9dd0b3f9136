"""Host checks of the jump driver's bookkeeping, with a stand-in solver on
the CPU: the fallback after a rejected jump (restore, plain cycle), the
deeper fallback when a divergence seeded by an earlier accepted jump shows
only in the next cycle (restore the older checkpoint, two plain cycles), an
error when the plain run itself diverges, and
the whole-cell co-moving displacement with its carried remainder."""
import math

import numpy as np
import pytest
import torch

from paper_2012_06144_amd import surrogate


class FakeSolver:
    """Steps a counter.  A jump entered through set_macroscopic may plant a
    'divergence' that makes stats() raise once the state has advanced
    `delay` steps past the jump; saved states carry the counter and the
    planted divergence."""

    def __init__(self, seed_jumps=(), delay=0, bad_indicator_jumps=(), diverge_at=None):
        self.diverge_at = diverge_at
        self.device = torch.device("cpu")
        self.t = 0
        self.bomb = None
        self.bad = False
        self.jumps = 0
        self.seed_jumps = set(seed_jumps)
        self.bad_indicator_jumps = set(bad_indicator_jumps)
        self.delay = delay
        self.log = []

    # state
    def new_state_buffer(self):
        return torch.zeros(3, dtype=torch.float64)

    def save_state(self, buf):
        buf[0] = self.t
        buf[1] = -1 if self.bomb is None else self.bomb
        buf[2] = float(self.bad)

    def restore_state(self, buf):
        self.t = int(buf[0])
        self.bomb = None if buf[1] < 0 else int(buf[1])
        self.bad = bool(buf[2])
        self.log.append(("restore", self.t))

    # stepping and fields
    def step(self, n):
        self.t += n

    def macroscopic(self, out):
        out.fill_(float(self.t))

    def set_macroscopic(self, phi, u, p, keep_neq=False):
        self.jumps += 1
        if self.jumps in self.seed_jumps:
            self.bomb = self.t + self.delay
        self.bad = self.jumps in self.bad_indicator_jumps
        self.log.append(("jump", self.t))

    def reduce_mass(self):
        return 1.0

    def stats(self):
        if (self.bomb is not None and self.t >= self.bomb) or (self.diverge_at and self.t >= self.diverge_at):
            raise RuntimeError(f"non-finite state at step {self.t}")
        return {"mass": 1.0, "xi_eff": 4.0, "max_speed": 0.5 if self.bad else 0.01,
                "centroid": (8.0, 8.0, 8.0), "rise_velocity": 1e-3}


class Setup:
    nx, ny, nz = 16, 16, 16
    phi_L, phi_H = 0.0, 1.0
    walls_y = True
    xi = 4.0


@pytest.fixture(autouse=True)
def _host_only(monkeypatch):
    monkeypatch.setattr(surrogate.sg, "sg_mass_project", lambda *a, **k: None)
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)


def _run(solver, total, **kw):
    jc = surrogate.JumpConfig(K=10, relax=20, m=5, box=(8, 8, 8), **kw)
    return surrogate.run_with_jumps(None, solver, Setup(), total, jc, log=lambda *_: None, mode="persistence")


def test_accepted_jumps_advance_by_whole_cycles():
    sv = FakeSolver()
    r = _run(sv, 5 + 4 * 30)
    assert (r["accepted"], r["rejected"]) == (4, 0)
    assert [e["step"] for e in r["trajectory"]] == [0, 35, 65, 95, 125]
    # a jump skips K steps: the solver ran 5 + 4 * 20 steps
    assert sv.t == 5 + 4 * 20


def test_rejected_jump_is_replaced_by_a_plain_cycle():
    sv = FakeSolver(bad_indicator_jumps=(2,))
    r = _run(sv, 5 + 4 * 30)
    assert (r["accepted"], r["rejected"]) == (3, 1)
    assert [e["jump"] for e in r["trajectory"][1:]] == [True, False, True, True]
    # the second cycle started at 5 + 20 solver steps and was rerun with K + relax plain steps
    assert ("restore", 25) in sv.log
    assert sv.t == 5 + 3 * 20 + 30


def test_divergence_seeded_by_an_accepted_jump_falls_back_one_cycle_further():
    # the first jump (at solver step 5) passes its own check at step 25 but
    # diverges at step 30, inside the next cycle and in its plain rerun
    sv = FakeSolver(seed_jumps=(1,), delay=25)
    r = _run(sv, 5 + 4 * 30)
    steps = [e["step"] for e in r["trajectory"]]
    assert steps == [0, 35, 65, 95, 125]
    assert [e["jump"] for e in r["trajectory"][1:]] == [False, False, True, True]
    assert (r["accepted"], r["rejected"]) == (2, 2)
    # back to the checkpoint before the first jump, then two plain cycles
    assert ("restore", 5) in sv.log
    assert sv.t == 5 + 2 * 30 + 2 * 20


def test_divergence_of_the_plain_run_raises():
    # a state that diverges with or without jumps ends the run loudly
    sv = FakeSolver(diverge_at=40)
    with pytest.raises(RuntimeError, match="non-finite"):
        _run(sv, 5 + 4 * 30)


def test_whole_cell_shift_carries_the_remainder(monkeypatch):
    # a bubble moving at u_y = 0.013 cells/step: K = 100 steps give 1.3 cells,
    # rounded to whole cells with the remainder carried, so the running total
    # stays within half a cell of 1.3 k
    monkeypatch.setattr(surrogate, "_gas_moments", lambda *a: (np.array([32.0]), np.array([[3.5, 3.5, 3.5]]),
                                                               np.array([[0.0, 0.013, 0.0]])))
    st = torch.zeros((8, 8, 8, 5), dtype=torch.float32)
    mem = {}
    total, seen = 0.0, set()
    for k in range(1, 11):
        d = surrogate.comoving_shift(st, 1, (8, 8, 8), 100, memory=mem, whole_cells=True)[0]
        dy = float(d[1])
        assert dy == round(dy) and float(d[0]) == 0.0 and float(d[2]) == 0.0
        seen.add(dy)
        total += dy
        assert abs(total - 1.3 * k) <= 0.5 + 1e-9
    assert seen == {1.0, 2.0}
    d = surrogate.comoving_shift(st, 1, (8, 8, 8), 100, whole_cells=False)[0]
    assert math.isclose(float(d[1]), 1.3, rel_tol=1e-6)


def test_cycle_hook_sees_each_cycle_start_and_may_advance_and_restore():
    # the rollout data generation samples K plain steps from each cycle start
    # inside the hook and restores the saved state: the run must not change
    seen = []

    def hook(k, box, F_now, F_prev, backup):
        seen.append((k, sv.t, float(F_now.flatten()[0]), float(F_prev.flatten()[0])))
        sv.step(10)
        sv.restore_state(backup)

    sv = FakeSolver()
    jc = surrogate.JumpConfig(K=10, relax=20, m=5, box=(8, 8, 8))
    r = surrogate.run_with_jumps(None, sv, Setup(), 5 + 4 * 30, jc, log=lambda *_: None, mode="persistence",
                                 on_cycle=hook)
    assert [k for k, *_ in seen] == [0, 1, 2, 3]
    # solver steps at each cycle start (a jump skips K = 10 of each 30-step cycle), with the trend
    # fields of that moment: F_now at the cycle start, F_prev m = 5 steps before
    assert [t for _, t, _, _ in seen] == [5, 25, 45, 65]
    assert [(a, b) for _, _, a, b in seen] == [(5.0, 0.0), (25.0, 20.0), (45.0, 40.0), (65.0, 60.0)]
    assert (r["accepted"], r["rejected"]) == (4, 0) and sv.t == 5 + 4 * 20
