"""Learned fast-forward for the coupled LBM: a 3D convolutional encoder-decoder
that predicts the macroscopic state (phi, u, p) K steps ahead, trained on
snapshots the solver itself produces, and a jump driver that alternates one
prediction with plain LBM relaxation steps and falls back to the plain solver
when its indicators trip.

Every tensor operation runs in the gfx950 kernels of ``sg.h`` (BF16
activations and weights, FP32 accumulation on the matrix cores, FP32 master
weights and Adam state); torch only allocates device memory.

Network (4 levels, 32-128 channels, 3x3x3 convolutions, leaky ReLU):
    enc0 16->32->32 | pool | enc1 32->64->64 | pool | enc2 64->128->128 | pool
    bottom 128->128->128 | up, concat enc2 | dec2 256->128->128 | up, concat enc1
    | dec1 192->64->64 | up, concat enc0 | dec0 96->32->32 | out 32->32 (FP32)
The output's first 5 channels are the increment (state(t+K) - state(t)) /
scale_out; the input's first 5 channels are state(t) / scale_in.
"""
from __future__ import annotations

import dataclasses
import json
import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import sg

SLOPE = 0.1
C_IN = 16
C_OUT = 32
NCH = 5

# (name, c_in, c_out, activation)
LAYERS = [
    ("enc0a", 16, 32, 1), ("enc0b", 32, 32, 1),
    ("enc1a", 32, 64, 1), ("enc1b", 64, 64, 1),
    ("enc2a", 64, 128, 1), ("enc2b", 128, 128, 1),
    ("bot_a", 128, 128, 1), ("bot_b", 128, 128, 1),
    ("dec2a", 256, 128, 1), ("dec2b", 128, 128, 1),
    ("dec1a", 192, 64, 1), ("dec1b", 64, 64, 1),
    ("dec0a", 96, 32, 1), ("dec0b", 32, 32, 1),
    ("out", 32, 32, 0),
]


def flops_per_voxel() -> float:
    """Multiply-adds x 2 per full-resolution voxel of one forward pass."""
    lvl = {"enc0": 1, "enc1": 8, "enc2": 64, "bot_": 512, "dec2": 64, "dec1": 8, "dec0": 1, "out": 1}
    total = 0.0
    for name, ci, co, _ in LAYERS:
        total += 2.0 * 27 * ci * co / lvl[name[:4] if name != "out" else "out"]
    return total


class Net:
    """Parameters, activations and gradients of the encoder-decoder on one device."""

    def __init__(self, device="cuda:0", seed: int = 0):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        g = torch.Generator(device="cpu").manual_seed(seed)
        self.p = {}
        for name, ci, co, act in LAYERS:
            fan_in = 27 * ci
            std = math.sqrt(2.0 / ((1 + SLOPE ** 2) * fan_in)) if act else 1e-3 / math.sqrt(fan_in)
            w = torch.randn((27, co, ci), generator=g) * std
            if name == "out":
                w[:, NCH:, :] = 0.0            # unused output channels stay zero
            d = {"w": w.to(self.device, torch.float32).contiguous(),
                 "b": torch.zeros(co, device=self.device, dtype=torch.float32)}
            d["wt"] = torch.empty((27, co, ci), device=self.device, dtype=torch.bfloat16)
            d["wm"] = torch.empty((27, ci, co), device=self.device, dtype=torch.bfloat16)
            for k in ("w", "b"):
                d["g" + k] = torch.zeros_like(d[k])
                d["m" + k] = torch.zeros_like(d[k])
                d["v" + k] = torch.zeros_like(d[k])
            sg.sg_to_bf16(d["w"], d["wt"])
            self.p[name] = d
        self.scale_in = [1.0, 1e-2, 1e-2, 1e-2, 1e-4]
        self.scale_out = [1e-2, 1e-3, 1e-3, 1e-3, 1e-5]
        self.scale_trend = [1e-3, 1e-5, 1e-5, 1e-5, 1e-7]
        self.base = "comoving"          # baseline whose residual the network predicts (see jump_base)
        self.step_count = 0
        self._ws = None

    # ---- helpers -----------------------------------------------------------------
    def _empty(self, shape, dtype=None):
        t = self.torch
        return t.empty(shape, device=self.device, dtype=dtype or t.bfloat16)

    def _conv(self, name, x, f32_out=False):
        d = self.p[name]
        _, ci, co, act = next(l for l in LAYERS if l[0] == name)
        assert x.shape[-1] == ci, (name, x.shape, ci)
        y = self._empty(x.shape[:-1] + (co,), self.torch.float32 if f32_out else None)
        sg.sg_conv3d_fwd(x, d["wt"], d["b"], co, co, act, SLOPE, y, int(f32_out))
        return y

    def _conv_up_cat(self, name, low, skip):
        """The layer applied to [up2(low), skip] without forming that tensor."""
        d = self.p[name]
        _, ci, co, act = next(l for l in LAYERS if l[0] == name)
        assert low.shape[-1] + skip.shape[-1] == ci, (name, low.shape, skip.shape, ci)
        y = self._empty(skip.shape[:-1] + (co,))
        sg.sg_conv3d_fwd_up_cat(low, skip, d["wt"], d["b"], co, co, act, SLOPE, y, 0)
        return y

    def _pool(self, x):
        n, dd, h, w, c = x.shape
        y = self._empty((n, dd // 2, h // 2, w // 2, c))
        sg.sg_pool2_fwd(x, y)
        return y

    def _up(self, x):
        n, dd, h, w, c = x.shape
        y = self._empty((n, 2 * dd, 2 * h, 2 * w, c))
        sg.sg_up2_fwd(x, y)
        return y

    def _cat(self, a, b):
        y = self._empty(a.shape[:-1] + (a.shape[-1] + b.shape[-1],))
        sg.sg_concat(a, b, y)
        return y

    # ---- forward -------------------------------------------------------------------
    def forward(self, x, keep=True):
        """x: (N, D, H, W, 16) BF16 with D, H, W divisible by 8 -> (N, D, H, W, 32) FP32."""
        a = {}
        a["x"] = x
        a["e0a"] = self._conv("enc0a", x)
        a["s0"] = self._conv("enc0b", a["e0a"])
        a["p1"] = self._pool(a["s0"])
        a["e1a"] = self._conv("enc1a", a["p1"])
        a["s1"] = self._conv("enc1b", a["e1a"])
        a["p2"] = self._pool(a["s1"])
        a["e2a"] = self._conv("enc2a", a["p2"])
        a["s2"] = self._conv("enc2b", a["e2a"])
        a["p3"] = self._pool(a["s2"])
        a["ba"] = self._conv("bot_a", a["p3"])
        a["bb"] = self._conv("bot_b", a["ba"])
        # the decoder's inputs [up2(coarse), skip] are formed only when the
        # backward pass needs them; inference reads both parts directly
        if keep:
            a["c2"] = self._cat(self._up(a["bb"]), a["s2"])
            a["d2a"] = self._conv("dec2a", a["c2"])
        else:
            a["d2a"] = self._conv_up_cat("dec2a", a["bb"], a["s2"])
        a["t2"] = self._conv("dec2b", a["d2a"])
        if keep:
            a["c1"] = self._cat(self._up(a["t2"]), a["s1"])
            a["d1a"] = self._conv("dec1a", a["c1"])
        else:
            a["d1a"] = self._conv_up_cat("dec1a", a["t2"], a["s1"])
        a["t1"] = self._conv("dec1b", a["d1a"])
        if keep:
            a["c0"] = self._cat(self._up(a["t1"]), a["s0"])
            a["d0a"] = self._conv("dec0a", a["c0"])
        else:
            a["d0a"] = self._conv_up_cat("dec0a", a["t1"], a["s0"])
        a["t0"] = self._conv("dec0b", a["d0a"])
        out = self._conv("out", a["t0"], f32_out=True)
        if keep:
            self.acts = a
        else:
            self.acts = None
        return out

    # ---- backward ------------------------------------------------------------------
    def _ws_for(self, x, co):
        n, d, h, w, ci = x.shape
        need = sg.sg_bwd_weight_workspace(n, d, h, w, ci, co)
        if self._ws is None or self._ws.numel() * 4 < need:
            self._ws = self._empty((need // 4 + 1,), self.torch.float32)
        return self._ws

    def _conv_bwd(self, name, x, y, dy, need_dx=True):
        """dy: gradient w.r.t. the layer output y; returns the gradient w.r.t. x."""
        d = self.p[name]
        _, ci, co, act = next(l for l in LAYERS if l[0] == name)
        if act:
            dp = self._empty(dy.shape)
            sg.sg_leaky_bwd(y, dy, dp, SLOPE)
        else:
            dp = dy
        sg.sg_conv3d_bwd_weight(x, dp, d["gw"], d["gb"], self._ws_for(x, co))
        if not need_dx:
            return None
        dx = self._empty(x.shape)
        sg.sg_conv3d_bwd_data(dp, d["wt"], dx, d["wm"])
        return dx

    def _split(self, g, ca, cb):
        a = self._empty(g.shape[:-1] + (ca,))
        b = self._empty(g.shape[:-1] + (cb,))
        sg.sg_split(g, ca, cb, a, b)
        return a, b

    def _up_bwd(self, g):
        n, dd, h, w, c = g.shape
        dx = self._empty((n, dd // 2, h // 2, w // 2, c))
        sg.sg_up2_bwd(g, dx)
        return dx

    def _pool_bwd(self, g, like):
        dx = self._empty(like.shape)
        sg.sg_pool2_bwd(g, dx)
        return dx

    def _add(self, a, b):
        y = self._empty(a.shape)
        sg.sg_add(a, b, y)
        return y

    def backward(self, dout):
        """dout: BF16 gradient of the loss w.r.t. the FP32 output (32 channels)."""
        a = self.acts
        g_t0 = self._conv_bwd("out", a["t0"], None, dout)
        g_d0a = self._conv_bwd("dec0b", a["d0a"], a["t0"], g_t0)
        g_c0 = self._conv_bwd("dec0a", a["c0"], a["d0a"], g_d0a)
        g_u0, g_s0 = self._split(g_c0, 64, 32)
        g_t1 = self._up_bwd(g_u0)
        g_d1a = self._conv_bwd("dec1b", a["d1a"], a["t1"], g_t1)
        g_c1 = self._conv_bwd("dec1a", a["c1"], a["d1a"], g_d1a)
        g_u1, g_s1 = self._split(g_c1, 128, 64)
        g_t2 = self._up_bwd(g_u1)
        g_d2a = self._conv_bwd("dec2b", a["d2a"], a["t2"], g_t2)
        g_c2 = self._conv_bwd("dec2a", a["c2"], a["d2a"], g_d2a)
        g_u2, g_s2 = self._split(g_c2, 128, 128)
        g_bb = self._up_bwd(g_u2)
        g_ba = self._conv_bwd("bot_b", a["ba"], a["bb"], g_bb)
        g_p3 = self._conv_bwd("bot_a", a["p3"], a["ba"], g_ba)
        g_s2 = self._add(g_s2, self._pool_bwd(g_p3, a["s2"]))
        g_e2a = self._conv_bwd("enc2b", a["e2a"], a["s2"], g_s2)
        g_p2 = self._conv_bwd("enc2a", a["p2"], a["e2a"], g_e2a)
        g_s1 = self._add(g_s1, self._pool_bwd(g_p2, a["s1"]))
        g_e1a = self._conv_bwd("enc1b", a["e1a"], a["s1"], g_s1)
        g_p1 = self._conv_bwd("enc1a", a["p1"], a["e1a"], g_e1a)
        g_s0 = self._add(g_s0, self._pool_bwd(g_p1, a["s0"]))
        g_e0a = self._conv_bwd("enc0b", a["e0a"], a["s0"], g_s0)
        self._conv_bwd("enc0a", a["x"], a["e0a"], g_e0a, need_dx=False)

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step_count += 1
        for name, d in self.p.items():
            sg.sg_adam(d["w"], d["gw"], d["mw"], d["vw"], d["wt"], lr, beta1, beta2, eps, self.step_count)
            sg.sg_adam(d["b"], d["gb"], d["mb"], d["vb"], None, lr, beta1, beta2, eps, self.step_count)

    def n_params(self) -> int:
        return sum(d["w"].numel() + d["b"].numel() for d in self.p.values())

    # ---- persistence -----------------------------------------------------------------
    def state_dict(self) -> dict:
        return {"w": {k: d["w"].cpu() for k, d in self.p.items()},
                "b": {k: d["b"].cpu() for k, d in self.p.items()},
                "scale_in": self.scale_in, "scale_out": self.scale_out, "steps": self.step_count}

    def load_state_dict(self, st):
        for k, d in self.p.items():
            d["w"].copy_(st["w"][k].to(self.device))
            d["b"].copy_(st["b"][k].to(self.device))
            sg.sg_to_bf16(d["w"], d["wt"])
        self.scale_in = list(st["scale_in"])
        self.scale_out = list(st["scale_out"])
        self.step_count = int(st["steps"])


# ---------------------------------------------------------------------------------------
# training data from the solver
# ---------------------------------------------------------------------------------------

@dataclass
class DataConfig:
    """Rising-bubble runs on an nx x ny x nz grid with seeded diameter, Eotvos
    number and centre offset.  Snapshots of (phi, u, p) every `every` steps
    from step `start`; `pairs_per_run` samples per run, each the triplet of
    states (t - m, t, t + K) cropped to `box` cells with the window centred
    on the bubble at t - m (the same window for all three)."""
    n_runs: int = 200
    grid: tuple = (128, 256, 128)
    d_range: tuple = (16.0, 40.0)
    eo_range: tuple = (2.0, 20.0)
    offset: float = 8.0
    centre_y: float = 80.0
    steps: int = 6000
    start: int = 400
    every: int = 50
    K: int = 200
    m: int = 25                    # steps between the two states the trend is taken from
    pairs_per_run: int = 10
    box: tuple = (80, 96, 80)      # (bx, by, bz), each divisible by 8
    seed: int = 7
    storage: str = "f32"


def _window(cent, box, grid):
    bx, by, bz = box
    nx, ny, nz = grid
    y0 = int(min(max(round(cent[1]) - by // 2, 1), ny - 1 - by))
    return (int(round(cent[0])) - bx // 2, y0, int(round(cent[2])) - bz // 2, bx, by, bz)


class _Stepper:
    """Advances a solver to absolute step counts."""

    def __init__(self, solver):
        self.sv, self.t = solver, 0

    def to(self, t):
        assert t >= self.t
        if t > self.t:
            self.sv.step(t - self.t)
            self.t = t


def generate_snapshots(cfg: DataConfig, device="cuda:0", log=print):
    """Runs the solver and returns the FP32 crops Sm, S0, S1 (samples,
    bz*by*bx*5, channels last) of the states at t - m, t and t + K on the
    device, the run index of every sample and the run parameters."""
    import torch

    from . import inputs, lbm
    rng = np.random.default_rng(cfg.seed)
    nx, ny, nz = cfg.grid
    bx, by, bz = cfg.box
    V = bx * by * bz
    nsnap = (cfg.steps - cfg.start) // cfg.every + 1
    lag = cfg.K // cfg.every
    assert lag * cfg.every == cfg.K and nsnap > lag and 0 < cfg.m <= cfg.start
    npr = min(cfg.pairs_per_run, nsnap - lag)
    ks = sorted(set(np.linspace(0, nsnap - lag - 1, npr).round().astype(int).tolist()))
    total = cfg.n_runs * len(ks)
    Sm = torch.empty((total, V * NCH), device=device, dtype=torch.float32)
    S0, S1 = torch.empty_like(Sm), torch.empty_like(Sm)
    xb = torch.empty(V * C_IN, device=device, dtype=torch.bfloat16)
    one = [1.0] * NCH
    run_of, meta = [], []
    slot = 0
    t0 = time.perf_counter()
    for r in range(cfg.n_runs):
        D = float(rng.uniform(*cfg.d_range))
        eo = float(rng.uniform(*cfg.eo_range))
        off = rng.uniform(-cfg.offset, cfg.offset, 3)
        g = eo * 1e-4 / (1.0 * D * D)          # Eo = g rho_H D^2 / sigma, sigma = 1e-4, rho_H = 1
        c = (nx / 2 + off[0], cfg.centre_y + off[1], nz / 2 + off[2])
        s = inputs.rising_bubble(nx, ny, nz, D=D, center=c, g=g)
        phi, u, ps = inputs.build_fields(s)
        sv = lbm.Solver(s.physics(), storage=cfg.storage, device=device)
        sv.init_fields(phi, u, ps)
        st = _Stepper(sv)
        y_first = None
        # the three states of each sample, in time order (samples may overlap)
        events = []
        for j, k in enumerate(ks):
            t = cfg.start + k * cfg.every
            events += [(t - cfg.m, 0, j), (t, 1, j), (t + cfg.K, 2, j)]
        boxes = {}
        for t, kind, j in sorted(events):
            st.to(t)
            if kind == 0:
                cent = sv.stats()["centroid"]
                if y_first is None:
                    y_first = cent[1]
                boxes[j] = _window(cent, cfg.box, cfg.grid)
            f = sv.macroscopic(torch.float32)
            dst = (Sm, S0, S1)[kind][slot + j]
            sg.sg_fields_to_input(*f, nx, ny, nz, boxes[j], one, C_IN, xb, dst)
            del f
        run_of += [r] * len(ks)
        slot += len(ks)
        y_last = sv.stats()["centroid"][1]
        meta.append({"D": D, "Eo": eo, "g": g, "centre": [float(v) for v in c]})
        log(f"[data] run {r}: D={D:.1f} Eo={eo:.1f}: {len(ks)} samples, rise {y_last - y_first:.2f} cells "
            f"({time.perf_counter() - t0:.0f}s)")
        del sv
    torch.cuda.synchronize()
    return Sm[:slot], S0[:slot], S1[:slot], np.array(run_of), meta


@dataclass
class RolloutConfig:
    """Training states taken from the jump driver itself: rising-bubble runs
    (seeded diameter, Eotvos number and centre offset) advanced by the
    driver with the co-moving trend jump; at every sampled cycle the states
    m steps before the cycle start and at it (the jump's inputs) are cropped
    to the driver's window, and the target is the state after K plain LBM
    steps from the cycle start, after which the driver resumes from its
    saved state.  The network so learns the residual of the baseline on the
    states it meets in the driver, which relaxed after earlier jumps."""
    n_runs: int = 30
    grid: tuple = (192, 640, 192)
    d_range: tuple = (32.0, 48.0)
    eo_range: tuple = (6.0, 14.0)
    offset: float = 8.0
    centre_y: float = 160.0
    warmup: int = 4000
    K: int = 100
    relax: int = 250
    m: int = 200
    cycles: int = 20
    first_sample: int = 2          # first sampled cycle (the first ones follow the start-up)
    box: tuple = (112, 128, 112)
    seed: int = 11
    storage: str = "f32"


def generate_rollout_snapshots(cfg: RolloutConfig, device="cuda:0", log=print):
    """Sm, S0, S1 crops (see RolloutConfig) on the device, the run index of
    every sample and the run parameters."""
    import torch

    from . import inputs, lbm
    rng = np.random.default_rng(cfg.seed)
    nx, ny, nz = cfg.grid
    bx, by, bz = cfg.box
    V = bx * by * bz
    per_run = cfg.cycles - cfg.first_sample
    total = cfg.n_runs * per_run
    Sm = torch.empty((total, V * NCH), device=device, dtype=torch.float32)
    S0, S1 = torch.empty_like(Sm), torch.empty_like(Sm)
    xb = torch.empty(V * C_IN, device=device, dtype=torch.bfloat16)
    one = [1.0] * NCH
    run_of, meta = [], []
    slot = 0
    t0 = time.perf_counter()
    for r in range(cfg.n_runs):
        D = float(rng.uniform(*cfg.d_range))
        eo = float(rng.uniform(*cfg.eo_range))
        off = rng.uniform(-cfg.offset, cfg.offset, 3)
        g = eo * 1e-4 / (1.0 * D * D)          # Eo = g rho_H D^2 / sigma, sigma = 1e-4, rho_H = 1
        c = (nx / 2 + off[0], cfg.centre_y + off[1], nz / 2 + off[2])
        s = inputs.rising_bubble(nx, ny, nz, D=D, center=c, g=g)
        phi, u, ps = inputs.build_fields(s)
        sv = lbm.Solver(s.physics(), storage=cfg.storage, device=device)
        sv.init_fields(phi, u, ps)
        jc = JumpConfig(K=cfg.K, relax=cfg.relax, m=cfg.m, warmup=cfg.warmup, box=cfg.box)
        start = slot

        def sample(k, box, F_now, F_prev, backup):
            nonlocal slot
            if k < cfg.first_sample or slot - start >= per_run:
                return
            sg.sg_fields_to_input(F_prev[0], F_prev[1:4], F_prev[4], nx, ny, nz, box, one, C_IN, xb, Sm[slot])
            sg.sg_fields_to_input(F_now[0], F_now[1:4], F_now[4], nx, ny, nz, box, one, C_IN, xb, S0[slot])
            sv.step(cfg.K)
            f = sv.macroscopic(torch.float32)
            sg.sg_fields_to_input(*f, nx, ny, nz, box, one, C_IN, xb, S1[slot])
            del f
            sv.restore_state(backup)
            slot += 1

        steps = cfg.warmup + cfg.m + cfg.cycles * (cfg.K + cfg.relax)
        run_with_jumps(None, sv, s, steps, jc, log=lambda *_: None, mode="comoving_trend", on_cycle=sample)
        run_of += [r] * (slot - start)
        meta.append({"D": D, "Eo": eo, "g": g, "centre": [float(v) for v in c]})
        log(f"[data] rollout run {r}: D={D:.1f} Eo={eo:.1f}: {slot - start} samples ({time.perf_counter() - t0:.0f}s)")
        del sv
        torch.cuda.empty_cache()
    torch.cuda.synchronize()
    return Sm[:slot], S0[:slot], S1[:slot], np.array(run_of), meta


def _moments(a, rows, scratch, out):
    sg.sg_channel_moments(a, rows, NCH, out, scratch)
    m = out.tolist()
    mean = [m[c] / rows for c in range(NCH)]
    var = [max(m[8 + c] / rows - mean[c] ** 2, 0.0) for c in range(NCH)]
    rms = [math.sqrt(m[8 + c] / rows) for c in range(NCH)]
    return mean, var, rms


PHI_HEAVY, PHI_LIGHT = 1.0, 0.0      # phase-field values of liquid and gas in the rising-bubble runs


def _gas_moments(states, count, box, phi_heavy, phi_light):
    """Gas volume, centroid (box coordinates) and gas-weighted velocity
    sum(chi u) / sum(chi) of each of `count` box states (sg_box_moments,
    FP64), as numpy arrays."""
    import torch
    bx, by, bz = box
    mom = torch.empty(count * 8, device=states.device, dtype=torch.float64)
    sg.sg_box_moments(states, count, bx, by, bz, phi_heavy, phi_light, mom)
    M = mom.view(count, 8).cpu().numpy()
    vol = M[:, 0]
    inv = 1.0 / np.maximum(vol, 1e-30)[:, None]
    return vol, M[:, 1:4] * inv, M[:, 4:7] * inv


def comoving_shift(states, count, box, K, prev=None, m=None, phi_heavy=PHI_HEAVY, phi_light=PHI_LIGHT,
                   max_gain=0.02, velocity="gas", memory=None, smooth=1.0, whole_cells=False):
    """Co-moving jump of each of `count` box states (contiguous, 5 FP32
    channels per voxel) over K steps.  velocity="gas": the bubble's
    gas-weighted velocity U and, given the same boxes `prev` m steps
    earlier, its acceleration a = (U - U_prev) / m give the displacement
    d = K U + K^2 a / 2 (the acceleration term at most K |U| / 2) and the
    velocity factor f = 1 + K a.U / |U|^2 (the flow around the bubble keeps
    its shape and grows with U), f clipped to 1 +- max_gain.
    velocity="centroid": U is the displacement of the gas centroid since
    `prev` over m, and f = 1.  With a dict `memory` (kept by the caller
    between calls on the same boxes) the acceleration is smoothed over calls,
    a <- smooth a + (1 - smooth) a_previous.  With whole_cells the
    displacement is rounded to whole cells, so the translation copies values
    instead of interpolating them (trilinear interpolation at a fractional
    shift s smooths every field by about s (1 - s) / 2 cell^2 per jump); the
    rounding remainder is carried in `memory` to the next call, so the
    displacements add up to the unrounded ones within half a cell.  Returns a
    (count, 4) FP32 device tensor of rows (dx, dy, dz, f); a box without gas
    stays put."""
    import torch
    vol, cen, U = _gas_moments(states, count, box, phi_heavy, phi_light)
    a = np.zeros_like(U)
    if prev is not None:
        vol_p, cen_p, Up = _gas_moments(prev, count, box, phi_heavy, phi_light)
        has = (vol_p > 0.5)[:, None]
        if velocity == "centroid":
            U = np.where(has, (cen - cen_p) / float(m), U)
        else:
            a = np.where(has, (U - Up) / float(m), 0.0)
    if memory is not None:
        if "a" in memory and memory["a"].shape == a.shape:
            a = smooth * a + (1.0 - smooth) * memory["a"]
        memory["a"] = a
    acc = 0.5 * K * K * a
    lim = 0.5 * K * np.linalg.norm(U, axis=1, keepdims=True)
    nacc = np.linalg.norm(acc, axis=1, keepdims=True)
    acc = np.where(nacc > lim, acc * lim / np.maximum(nacc, 1e-300), acc)
    d = K * U + acc
    if whole_cells:
        if memory is not None and "carry" in memory and memory["carry"].shape == d.shape:
            d = d + memory["carry"]
        r = np.round(d)
        if memory is not None:
            memory["carry"] = d - r
        d = r
    uu = (U * U).sum(1)
    f = 1.0 + K * np.where(uu > 0, (a * U).sum(1) / np.maximum(uu, 1e-300), 0.0)
    f = np.clip(f, 1.0 - max_gain, 1.0 + max_gain)
    out = np.concatenate([d, f[:, None]], axis=1)
    out[vol <= 0.5] = (0.0, 0.0, 0.0, 1.0)
    return torch.from_numpy(out.astype(np.float32)).to(states.device)


def bubble_frame_shifts(s0, sm, box, K, m, phi_heavy=PHI_HEAVY, phi_light=PHI_LIGHT):
    """Displacements of the co-moving trend jump of one box state s0, given
    the same box m steps earlier (sm): the bubble's gas-weighted velocities U
    and U_m give its displacement over the trend window, m (U + U_m) / 2,
    and over the jump, K U + K^2 a / 2 with a = (U - U_m) / m (the
    acceleration term at most K |U| / 2).  Returns two (4,) FP32 device
    tensors (dx, dy, dz, 1) for sg_shift_boxes (velocity factor 1)."""
    import torch
    vol, _, U = _gas_moments(s0, 1, box, phi_heavy, phi_light)
    vol_m, _, Um = _gas_moments(sm, 1, box, phi_heavy, phi_light)
    if vol[0] <= 0.5 or vol_m[0] <= 0.5:
        U = Um = np.zeros((1, 3))
    a = (U[0] - Um[0]) / float(m)
    acc = 0.5 * K * K * a
    lim = 0.5 * K * np.linalg.norm(U[0])
    if np.linalg.norm(acc) > lim:
        acc = acc * lim / np.linalg.norm(acc)
    d_m = 0.5 * m * (U[0] + Um[0])
    d_k = K * U[0] + acc
    mk = lambda d: torch.tensor([d[0], d[1], d[2], 1.0], dtype=torch.float32).to(s0.device)
    return mk(d_m), mk(d_k)


def comoving_trend_base(s0, sm, box, K, m, phi_lo, phi_hi, u_by_phase, out, phi_heavy=PHI_HEAVY,
                        phi_light=PHI_LIGHT, gain=1.0):
    """Co-moving trend jump: the state's development in the bubble's frame is
    extrapolated (a projective step, Gear and Kevrekidis 2003, taken in the
    frame that moves with the bubble), then the result is translated with
    the bubble:
      s(t + K) = T_dK[ s(t) + (K/m) (s(t) - T_dm[s(t - m)]) ],
    T_d being the window translation by d (sg_shift_boxes) and dm, dK the
    displacements of bubble_frame_shifts.  Unlike the plain co-moving jump
    this follows the growth of the wake, not only the growth of the
    velocity.  phi is only translated (extrapolating its trend thinned the
    interface over many cycles) and the pressure is carried over;
    u_by_phase weights the velocity trend by the heavy-phase fraction (1) or
    by the bulk of the heavy phase only (2), and `gain` scales K/m
    (sg_projective_step)."""
    import torch
    bx, by, bz = box
    d_m, d_k = bubble_frame_shifts(s0, sm, box, K, m, phi_heavy, phi_light)
    moved = torch.empty_like(s0)
    sg.sg_shift_boxes(sm, 1, bx, by, bz, d_m, moved)
    ext = torch.empty_like(s0)
    sg.sg_projective_step(s0, moved, bx * by * bz, 1, 5, gain * K / m, phi_lo, phi_hi, int(u_by_phase), 0, 0, ext)
    sg.sg_shift_boxes(ext, 1, bx, by, bz, d_k, out)


def jump_base(kind, s0, box, K, out, shift=None):
    """Baseline state K steps ahead of one box state s0 (into out):
    "transport": phi moved by the local velocity (semi-Lagrangian), u and p
    carried over; "comoving": every channel translated with the bubble and
    the velocity scaled (`shift`, a (4,) device tensor from comoving_shift:
    the exact jump of a bubble rising steadily, followed to first order
    while it accelerates)."""
    bx, by, bz = box
    if kind == "comoving":
        sg.sg_shift_boxes(s0, 1, bx, by, bz, shift, out)
    else:
        sg.sg_advect_phase(s0, 1, bx, by, bz, K, out)


def _base_crop(S0, i, box, K, out, base, shifts, Sm=None, m=None):
    """Baseline of sample i; the co-moving displacement comes from `shifts`
    (all samples, comoving_shift) or is measured on the sample itself (and
    its state m steps earlier, Sm[i]); the co-moving trend baseline takes
    Sm[i] as its trend state."""
    if base == "comoving_trend":
        comoving_trend_base(S0[i], Sm[i], box, K, m, PHI_LIGHT, PHI_HEAVY, 1, out)
        return
    if base == "comoving" and shifts is None:
        shift = comoving_shift(S0[i], 1, box, K, prev=None if Sm is None else Sm[i], m=m)[0]
    else:
        shift = None if shifts is None else shifts[i]
    jump_base(base, S0[i], box, K, out, shift)


def channel_scales(Sm, S0, S1, box, K, m, base_kind="comoving", shifts=None):
    """Per-channel input scale (root mean square of the state; 1 for phi),
    output scale (standard deviation of the target S1 - baseline, the
    baseline of kind `base_kind`, see jump_base) and trend scale (root mean
    square of S(t) - S(t - m)), over all samples.  FP64 moments from
    sg_channel_moments."""
    import torch
    bx, by, bz = box
    V = bx * by * bz
    n = S0.shape[0]
    out = torch.zeros(16, device=S0.device, dtype=torch.float64)
    scratch = torch.zeros(512 * 16, device=S0.device, dtype=torch.float64)
    _, _, rms = _moments(S0, n * V, scratch, out)
    sin = [1.0] + [max(r, 1e-12) for r in rms[1:]]
    acc = np.zeros(16)
    tacc = np.zeros(16)
    base = torch.empty((V * NCH,), device=S0.device, dtype=torch.float32)
    diff = torch.empty((V * NCH,), device=S0.device, dtype=torch.float32)
    for i in range(n):
        _base_crop(S0, i, box, K, base, base_kind, shifts, Sm, m)
        sg.sg_make_target(base, S1[i], [1.0] * NCH, NCH, diff)
        sg.sg_channel_moments(diff, V, NCH, out, scratch)
        acc += out.cpu().numpy()
        sg.sg_make_target(Sm[i], S0[i], [1.0] * NCH, NCH, diff)
        sg.sg_channel_moments(diff, V, NCH, out, scratch)
        tacc += out.cpu().numpy()
    rows = n * V
    var = [max(acc[8 + c] / rows - (acc[c] / rows) ** 2, 0.0) for c in range(NCH)]
    sout = [max(math.sqrt(v), 1e-12) for v in var]
    strend = [max(math.sqrt(tacc[8 + c] / rows), 1e-12) for c in range(NCH)]
    return [float(v) for v in sin], [float(v) for v in sout], [float(v) for v in strend]


def trend_scale(net, K, m):
    """Input factor of the trend channels: (s - s_prev) over its root mean
    square in the training data."""
    return [1.0 / q for q in net.scale_trend]


def make_batch(net, Sm, S0, S1, idx, box, K, m, target_from="baseline", shifts=None):
    """Network input (BF16: state and its trend S0 - Sm, normalised) and
    target (FP32) of the samples `idx`.  The target is (S1 - base) /
    scale_out with base the network's baseline (net.base; `shifts` holds
    the co-moving displacements of all samples), the transport baseline
    with target_from="transport", or base = S0 (persistence) with
    target_from="state"."""
    import torch
    bx, by, bz = box
    V = bx * by * bz
    n = len(idx)
    x = torch.empty((n, bz, by, bx, C_IN), device=S0.device, dtype=torch.bfloat16)
    t = torch.empty((n, bz, by, bx, C_OUT), device=S0.device, dtype=torch.float32)
    base = torch.empty((V * NCH,), device=S0.device, dtype=torch.float32)
    ts = trend_scale(net, K, m)
    for j, i in enumerate(idx):
        sg.sg_pair_to_input(S0[i], Sm[i], net.scale_in, ts, C_IN, x[j])
        if target_from in ("baseline", "transport"):
            kind = net.base if target_from == "baseline" else "transport"
            _base_crop(S0, i, box, K, base, kind, shifts, Sm, m)
            sg.sg_make_target(base, S1[i], net.scale_out, C_OUT, t[j])
        else:
            sg.sg_make_target(S0[i], S1[i], net.scale_out, C_OUT, t[j])
    return x, t


def train(net, Sm, S0, S1, box, K, m, run_of=None, steps=500, batch=8, lr=2e-4, warmup=50, val_frac=0.1,
          seed=0, log=print, shifts=None):
    """Adam on the MSE of the normalised residual of the network's baseline,
    linear warm-up over `warmup` steps, then cosine learning-rate decay.
    Validation samples are whole runs held out (samples of one run are
    correlated).  Returns the loss history and the validation losses of the
    network, of its baseline alone, of the transport baseline and of
    persistence."""
    import torch
    n = S0.shape[0]
    rng = np.random.default_rng(seed)
    if run_of is None:
        run_of = np.arange(n)
    runs = np.unique(run_of)
    vr = rng.permutation(runs)[:max(1, int(round(val_frac * len(runs))))]
    val = np.nonzero(np.isin(run_of, vr))[0]
    tr = np.nonzero(~np.isin(run_of, vr))[0]
    loss = torch.zeros(1, device=S0.device, dtype=torch.float32)
    scratch = torch.zeros(1024, device=S0.device, dtype=torch.float32)
    hist = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(steps):
        idx = rng.choice(tr, size=min(batch, len(tr)), replace=False)
        x, t = make_batch(net, Sm, S0, S1, idx, box, K, m, shifts=shifts)
        out = net.forward(x)
        g = torch.empty(out.shape, device=out.device, dtype=torch.bfloat16)
        sg.sg_mse(out, t, loss, g, scratch)
        net.backward(g)
        cur_lr = lr * min(1.0, (it + 1) / max(1, warmup)) * 0.5 * (1 + math.cos(math.pi * it / steps))
        net.adam(cur_lr)
        if it % 50 == 0 or it == steps - 1:
            lv = float(loss.item())
            hist.append((it, lv))
            log(f"[train] step {it} loss {lv:.4e} ({time.perf_counter() - t0:.1f}s)")
            best = min(v for _, v in hist)
            if not math.isfinite(lv) or lv > 20.0 * best:
                lr *= 0.5                       # divergence guard: halve the rate from here on
                log(f"[train] loss rose to {lv:.3e} (best {best:.3e}): learning rate halved to {lr:.2e}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    v = evaluate(net, Sm, S0, S1, val, box, K, m, shifts=shifts)
    return {"history": hist, "val_loss": v["network"], "val_loss_baseline": v["baseline"],
            "val_loss_transport": v["transport"], "val_loss_persistence": v["persistence"], "seconds": wall,
            "base": net.base,
            "n_train": int(len(tr)), "n_val": int(len(val)), "val_runs": [int(v) for v in vr]}


def evaluate(net, Sm, S0, S1, idx, box, K, m, batch=8, shifts=None):
    """Mean validation MSE (normalised units) of the jump with the network
    (its baseline + network residual), of that baseline alone (network
    output 0), of the transport baseline and of persistence (state left
    unchanged)."""
    import torch
    loss = torch.zeros(1, device=S0.device, dtype=torch.float32)
    scratch = torch.zeros(1024, device=S0.device, dtype=torch.float32)
    tot = {"network": 0.0, "baseline": 0.0, "transport": 0.0, "persistence": 0.0}
    cnt = 0
    for k in range(0, len(idx), batch):
        ii = idx[k:k + batch]
        x, t = make_batch(net, Sm, S0, S1, ii, box, K, m, shifts=shifts)
        out = net.forward(x, keep=False)
        g = torch.empty(out.shape, device=out.device, dtype=torch.bfloat16)
        sg.sg_mse(out, t, loss, g, scratch)
        tot["network"] += float(loss.item()) * len(ii)
        zero = torch.zeros_like(out)
        sg.sg_mse(zero, t, loss, g, scratch)
        tot["baseline"] += float(loss.item()) * len(ii)
        for name in ("transport", "state"):
            _, tp = make_batch(net, Sm, S0, S1, ii, box, K, m, target_from=name, shifts=shifts)
            sg.sg_mse(zero, tp, loss, g, scratch)
            tot["transport" if name == "transport" else "persistence"] += float(loss.item()) * len(ii)
        cnt += len(ii)
    return {k: v / cnt for k, v in tot.items()}


# ---------------------------------------------------------------------------------------
# jump driver
# ---------------------------------------------------------------------------------------

@dataclass
class JumpConfig:
    K: int = 200                # steps one jump skips
    relax: int = 50             # LBM steps after each jump
    m: int = 25                 # the trend is taken over the last m relaxation steps (m <= relax), or
                                # between consecutive cycle ends (m = K + relax)
    mass_tol: float = 1e-6      # |d sum(phi)| / sum(phi) over a cycle
    xi_lo: float = 0.8          # interface width must stay in [xi_lo, xi_hi] * xi
    xi_hi: float = 1.25
    u_max: float = 0.05         # indicator: max |u| after the relaxation (lattice units)
    box: tuple = (112, 128, 112)  # network window around the bubble (bx, by, bz), divisible by 8
    predict_pressure: bool = False  # apply the network's pressure residual (else p follows the baseline)
    net_phi_only: bool = False  # apply only the network's phase-field residual (u follows the baseline)
    u_by_phase: bool = True     # weight velocity increments by the heavy-phase fraction
    phi_at_interface: bool = True  # weight phi increments by 4 q (1 - q): none in the bulk phases
    accel: bool = True          # co-moving jumps use the state of the trend window (acceleration or
                                # centroid displacement, see comoving_shift)
    velocity: str = "gas"       # bubble velocity of co-moving jumps: "gas" (gas-weighted u) or "centroid"
    max_gain: float = 0.02      # co-moving velocity factor limited to 1 +- max_gain
    accel_smooth: float = 1.0   # weight of the newest acceleration estimate (1: no smoothing)
    warmup: int = 0             # plain LBM steps before the first jump (the start-up from rest)
    clip_phi: bool = True       # clip the jumped phi to [phi_L, phi_H] (removes the phase field's own
                                # small over- and undershoots, which the mass projection then moves
                                # into the interface)
    whole_cells: bool = False   # co-moving displacement rounded to whole cells, remainder carried over
    trend_gain: float = 1.0     # co-moving trend jump: factor on the extrapolation ratio K/m
    trend_bulk: bool = False    # co-moving trend jump: velocity trend in the bulk of the heavy phase only
    keep_neq: bool = False      # after a jump keep the populations' non-equilibrium parts
                                # (lbm_shift_equilibrium) instead of rebuilding them at equilibrium;
                                # they stay at their cells while the interface moves, which
                                # destabilised long runs at a density ratio of 1000


def across_trend(jc) -> bool:
    """The trend is taken between consecutive cycle ends (m = K + relax)."""
    return jc.m == jc.K + jc.relax


def _traj_entry(step, st, **kw):
    d = {"step": step, "centroid_y": st["centroid"][1], "rise_velocity": st["rise_velocity"], "mass": st["mass"],
         "xi_eff": st["xi_eff"], "max_speed": st["max_speed"]}
    d.update(kw)
    return d


def _jump(net, mode, F_now, F_prev, setup, box, jc: JumpConfig, diagnostics=False, memory=None):
    """Writes the state K steps ahead into F_now ((5, nz, ny, nx) FP32 planes:
    phi, u, p) from F_now and F_prev (m steps earlier).  mode "persistence":
    unchanged; "transport": phi moved by the local velocity in the window
    around the bubble; "comoving": the window translated by K times the
    bubble's gas-weighted velocity; "projective": projective step over the
    whole grid; "network": the network's baseline (net.base) plus its
    residual (from the state and its trend) in the window."""
    import torch
    nx, ny, nz = setup.nx, setup.ny, setup.nz
    N = nx * ny * nz
    lo, hi = min(setup.phi_L, setup.phi_H), max(setup.phi_L, setup.phi_H)
    if mode == "persistence":
        return None
    if mode == "projective":
        sg.sg_projective_step(F_now, F_prev, N, N, 1, jc.K / jc.m, lo, hi, int(jc.u_by_phase), 1, 0, F_now)
        return None
    bx, by, bz = box[3], box[4], box[5]
    V = bx * by * bz
    one = [1.0] * NCH
    s0 = torch.empty(V * NCH, device=F_now.device, dtype=torch.float32)
    base = torch.empty_like(s0)
    x = torch.empty((1, bz, by, bx, C_IN), device=F_now.device, dtype=torch.bfloat16)
    sg.sg_fields_to_input(F_now[0], F_now[1:4], F_now[4], nx, ny, nz, box, one, C_IN, x, s0)
    kind = net.base if mode == "network" else mode
    sm = torch.empty_like(s0)
    sg.sg_fields_to_input(F_prev[0], F_prev[1:4], F_prev[4], nx, ny, nz, box, one, C_IN, x, sm)
    shift = None
    if kind == "comoving":
        shift = comoving_shift(s0, 1, (bx, by, bz), jc.K, prev=sm if jc.accel else None, m=jc.m,
                               phi_heavy=setup.phi_H, phi_light=setup.phi_L, max_gain=jc.max_gain,
                               velocity=jc.velocity, memory=memory, smooth=jc.accel_smooth,
                               whole_cells=jc.whole_cells)[0]
    if kind == "comoving_trend":
        assert not across_trend(jc), "the co-moving trend jump takes its trend inside the relaxation"
        comoving_trend_base(s0, sm, (bx, by, bz), jc.K, jc.m, lo, hi, 2 if jc.trend_bulk else int(jc.u_by_phase),
                            base, phi_heavy=setup.phi_H, phi_light=setup.phi_L, gain=jc.trend_gain)
    else:
        jump_base(kind, s0, (bx, by, bz), jc.K, base, shift)
    inc = None
    if mode == "network":
        sg.sg_pair_to_input(s0, sm, net.scale_in, trend_scale(net, jc.K, jc.m), C_IN, x)
        out = net.forward(x, keep=False)
        so = list(net.scale_out)
        if not jc.predict_pressure:
            so[4] = 0.0
        if jc.net_phi_only:
            so[1] = so[2] = so[3] = 0.0
    else:
        out = torch.zeros((V, C_OUT), device=F_now.device, dtype=torch.float32)
        so = [0.0] * NCH
    sg.sg_apply_prediction(out, C_OUT, so, F_now[0], F_now[1:4], F_now[4], nx, ny, nz, box,
                           int(setup.walls_y), lo, hi, base=base, u_by_phase=jc.u_by_phase,
                           phi_at_interface=jc.phi_at_interface, clip=jc.clip_phi)
    if diagnostics and mode == "network":
        mx = out.view(-1, C_OUT)[:, :NCH].abs().amax(0).tolist()
        inc = [float(a * b) for a, b in zip(mx, so)]
    return inc


def run_with_jumps(net, solver, setup, total_steps, jc: JumpConfig, log=print, mode="network", on_cycle=None):
    """Advances `solver` by total_steps: jc.warmup plain steps (the start-up
    from rest), m plain steps to start the trend,
    then cycles of one jump (K steps, see _jump) plus jc.relax LBM steps,
    the fields being taken m steps before the end of each relaxation and at
    its end.  After each cycle the indicators are checked (finite, mass drift
    over the cycle <= mass_tol, interface width in [xi_lo, xi_hi] xi, max |u|
    <= u_max); if one trips, the state saved before the jump is restored and
    the cycle's K + relax steps are run with the plain LBM.  If the state is
    still unusable after that (a divergence seeded by the previous, accepted
    jump), the state saved one cycle earlier is restored and both cycles are
    run plainly; a run that fails even then raises.  The jumped
    fields enter the solver through lbm_shift_equilibrium (populations keep
    their non-equilibrium parts) or, with jc.keep_neq False, are rebuilt at
    equilibrium.  on_cycle(k, box, F_now, F_prev, backup), if given, is
    called at the start of cycle k once its state is saved to `backup` and
    before the jump; it may advance the solver if it restores `backup`."""
    import torch
    nx, ny, nz = setup.nx, setup.ny, setup.nz
    shape = (5, nz, ny, nx)
    F_now = torch.empty(shape, device=solver.device, dtype=torch.float32)
    F_prev = torch.empty_like(F_now)
    backup = solver.new_state_buffer()
    older = solver.new_state_buffer()   # the state saved one cycle before `backup`
    have_older = False
    scratch = torch.zeros(2048, device=solver.device, dtype=torch.float64)
    cyc = jc.K + jc.relax
    accepted = rejected = 0
    traj = [_traj_entry(0, solver.stats())]
    t_jump = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_log = t0
    across = jc.m == cyc               # trend between consecutive cycle ends
    memory = {}                         # acceleration estimate carried between cycles
    cycle = 0
    assert across or 0 < jc.m <= jc.relax
    if jc.warmup:                       # plain steps before the first jump
        solver.step(jc.warmup)
        traj.append(_traj_entry(jc.warmup, solver.stats()))
    solver.macroscopic(out=F_prev)
    solver.step(jc.m)
    done = jc.warmup + jc.m
    solver.macroscopic(out=F_now)
    F_keep = torch.empty_like(F_now) if across else None

    def plain_cycle():
        # one cycle of plain steps, with the trend fields taken as a jump cycle takes them
        if across:
            solver.step(cyc)
        else:
            solver.step(cyc - jc.m)
            solver.macroscopic(out=F_prev)
            solver.step(jc.m)
        return solver.stats()

    while done + cyc <= total_steps:
        m0 = solver.reduce_mass()
        cent = solver.stats()["centroid"]
        if done > jc.warmup + jc.m:     # keep the previous cycle's start as the older checkpoint
            backup, older = older, backup
            have_older = True
        solver.save_state(backup)
        box = _window(cent, jc.box, (nx, ny, nz))
        if on_cycle is not None:
            on_cycle(cycle, box, F_now, F_prev, backup)
        cycle += 1
        tp = time.perf_counter()
        if across:
            F_keep.copy_(F_now)
        inc = _jump(net, mode, F_now, F_prev, setup, box, jc, diagnostics=len(traj) <= 4, memory=memory)
        sg.sg_mass_project(F_now[0], setup.walls_y, m0, min(setup.phi_L, setup.phi_H), max(setup.phi_L, setup.phi_H),
                           scratch)
        solver.set_macroscopic(F_now[0], F_now[1:4], F_now[4], keep_neq=jc.keep_neq)
        torch.cuda.synchronize()
        t_jump += time.perf_counter() - tp
        if across:
            F_prev, F_keep = F_keep, F_prev
            solver.step(jc.relax)
        else:
            if jc.relax > jc.m:
                solver.step(jc.relax - jc.m)
            solver.macroscopic(out=F_prev)
            solver.step(jc.m)
        try:
            st = solver.stats()
            drift = abs(st["mass"] - m0) / abs(m0)
            ok = (drift <= jc.mass_tol and jc.xi_lo * setup.xi <= st["xi_eff"] <= jc.xi_hi * setup.xi
                  and st["max_speed"] <= jc.u_max)
        except Exception as e:          # non-finite state after the jump
            st, drift, ok = None, float("nan"), False
            log(f"[jump] cycle at step {done}: {e}")
        if inc is not None:
            log(f"[jump] cycle at step {done}: max network residual {['%.2e' % v for v in inc]}, "
                f"drift {drift:.2e}, xi_eff {st['xi_eff'] if st else float('nan'):.3f}")
        if ok:
            accepted += 1
        else:
            rejected += 1
            solver.restore_state(backup)
            try:
                st = plain_cycle()
            except Exception as e:
                if not have_older:
                    raise
                log(f"[jump] cycle at step {done}: plain rerun failed ({e}); back to step {done - cyc}")
                solver.restore_state(older)
                if traj[-1].get("jump"):
                    accepted -= 1
                    rejected += 1
                traj[-1] = _traj_entry(done, plain_cycle(), jump=False, drift=float("nan"))
                if across:
                    solver.macroscopic(out=F_prev)
                st = plain_cycle()
                drift = float("nan")
        solver.macroscopic(out=F_now)
        done += cyc
        traj.append(_traj_entry(done, st, jump=bool(ok), drift=drift))
        if time.perf_counter() - t_log > 30.0:
            t_log = time.perf_counter()
            log(f"[jump] {mode} step {done}: centroid y {st['centroid'][1]:.3f}, {accepted} accepted, "
                f"{rejected} rejected")
    if done < total_steps:
        solver.step(total_steps - done)
        done = total_steps
        traj.append(_traj_entry(done, solver.stats()))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"[jump] {mode}: {accepted} accepted, {rejected} rejected, {wall:.1f}s ({t_jump:.2f}s in jumps)")
    return {"trajectory": traj, "accepted": accepted, "rejected": rejected, "seconds": wall,
            "seconds_jump": t_jump}


def run_plain(solver, total_steps, every, first=None, log=print):
    """The plain LBM with the statistics cadence of the jump driver: at step
    0, at `first`, then every `every` steps, and at the end."""
    import torch
    traj = [_traj_entry(0, solver.stats())]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    if first:
        solver.step(first)
        done = first
        traj.append(_traj_entry(done, solver.stats()))
    last_log = time.perf_counter()
    while done < total_steps:
        n = min(every, total_steps - done)
        solver.step(n)
        done += n
        traj.append(_traj_entry(done, solver.stats()))
        if time.perf_counter() - last_log > 30.0:
            last_log = time.perf_counter()
            log(f"[plain] step {done}: centroid y {traj[-1]['centroid_y']:.3f}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"[plain] {total_steps} steps, {wall:.1f}s")
    return {"trajectory": traj, "seconds": wall}


def compare_trajectories(ref, run):
    """Rise-velocity and centroid errors of `run` against `ref` at the steps
    both recorded.  The rise velocity is the gas-weighted u_y (the
    statistics' rise_velocity); its mean relative error over the second
    half is the headline figure.  The slope of the gas centroid is reported
    too, but the plain run's centroid wanders by a cell or more over a few
    thousand steps while the gas-weighted velocity stays smooth."""
    rs = {e["step"]: e for e in ref["trajectory"]}
    common = [e for e in run["trajectory"] if e["step"] in rs]
    steps = np.array([e["step"] for e in common], dtype=np.float64)
    y = np.array([e["centroid_y"] for e in common])
    yr = np.array([rs[e["step"]]["centroid_y"] for e in common])
    half = len(steps) // 2
    slope = np.polyfit(steps[half:], y[half:], 1)[0]
    slope_r = np.polyfit(steps[half:], yr[half:], 1)[0]
    ur = np.array([rs[e["step"]]["rise_velocity"] for e in common])
    uu = np.array([e["rise_velocity"] for e in common])
    return {"centroid_err_max_cells": float(np.max(np.abs(y - yr))),
            "centroid_err_final_cells": float(abs(y[-1] - yr[-1])),
            "rise_rel_err_centroid_slope": float(abs(slope - slope_r) / abs(slope_r)),
            "rise_rel_err_velocity_final": float(abs(uu[-1] - ur[-1]) / abs(ur[-1])),
            "rise_rel_err_velocity_max_2nd_half": float(np.max(np.abs(uu[half:] - ur[half:])) / np.max(np.abs(ur[half:]))),
            "rise_rel_err_velocity_mean_2nd_half": float(np.mean(np.abs(uu[half:] - ur[half:])) /
                                                         np.mean(np.abs(ur[half:]))),
            "rise_ref_cells": float(yr[-1] - yr[0])}


# ---------------------------------------------------------------------------------------
# persistence and command line
# ---------------------------------------------------------------------------------------

def save_weights(net, path):
    """FP32 master weights, biases and the normalisation scales (safetensors)."""
    from safetensors.torch import save_file
    t = {}
    for k, d in net.p.items():
        t[k + ".w"] = d["w"].detach().cpu().contiguous()
        t[k + ".b"] = d["b"].detach().cpu().contiguous()
    meta = {"scale_in": json.dumps(net.scale_in), "scale_out": json.dumps(net.scale_out),
            "scale_trend": json.dumps(net.scale_trend), "steps": str(net.step_count), "base": net.base}
    save_file(t, path, metadata=meta)


def load_weights(net, path):
    from safetensors import safe_open
    with safe_open(path, framework="pt") as f:
        meta = f.metadata()
        for k, d in net.p.items():
            d["w"].copy_(f.get_tensor(k + ".w").to(d["w"].device))
            d["b"].copy_(f.get_tensor(k + ".b").to(d["b"].device))
            sg.sg_to_bf16(d["w"], d["wt"])
    net.scale_in = json.loads(meta["scale_in"])
    net.scale_out = json.loads(meta["scale_out"])
    net.scale_trend = json.loads(meta["scale_trend"])
    net.step_count = int(meta["steps"])
    net.base = meta.get("base", "transport")


def _cmd_train(a):
    import torch
    if a.rollout:
        cfg = RolloutConfig(n_runs=a.runs, K=a.K, m=a.m, relax=a.relax, cycles=a.cycles)
        if a.box:
            cfg.box = tuple(int(v) for v in a.box.split("x"))
    else:
        cfg = DataConfig(n_runs=a.runs, steps=a.lbm_steps, pairs_per_run=a.pairs_per_run, m=a.m, K=a.K)
    t0 = time.perf_counter()
    Sm, S0, S1, run_of, meta = (generate_rollout_snapshots if a.rollout else generate_snapshots)(cfg, log=_log)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    net = Net(seed=a.seed)
    net.base = a.base
    shifts = (comoving_shift(S0, S0.shape[0], cfg.box, cfg.K, prev=Sm, m=cfg.m, whole_cells=a.whole_cells)
              if a.base == "comoving" else None)
    net.scale_in, net.scale_out, net.scale_trend = channel_scales(Sm, S0, S1, cfg.box, cfg.K, cfg.m,
                                                                  base_kind=a.base, shifts=shifts)
    res = train(net, Sm, S0, S1, cfg.box, cfg.K, cfg.m, run_of=run_of, steps=a.train_steps, batch=a.batch,
                lr=a.lr, log=_log, shifts=shifts)
    res.update({"data_seconds": t_data, "samples": int(S0.shape[0]), "runs": meta, "config": cfg.__dict__,
                "scale_in": net.scale_in, "scale_out": net.scale_out, "scale_trend": net.scale_trend,
                "params": net.n_params()})
    _log(f"[train] val loss {res['val_loss']:.4e}; {a.base} baseline alone {res['val_loss_baseline']:.4e}; "
         f"transport {res['val_loss_transport']:.4e}; persistence {res['val_loss_persistence']:.4e}")
    if a.weights:
        save_weights(net, a.weights)
    return res


def _cmd_jump(a):
    import torch

    from . import inputs, lbm
    s = inputs.surrogate_jump_bubble(steps=a.steps)
    if a.grid:
        nx, ny, nz = (int(v) for v in a.grid.split("x"))
        D = a.D if a.D else s.radius * 2
        g = a.eo * 1e-4 / (D * D)          # Eo = g rho_H D^2 / sigma, sigma = 1e-4, rho_H = 1
        s = inputs.rising_bubble(nx, ny, nz, D=D, center=(nx / 2, ny / 4, nz / 2), g=g, steps=a.steps)
        s.name = f"rising_bubble_{nx}x{ny}x{nz}_D{D:g}_Eo{a.eo:g}"
    phi, u, ps = inputs.build_fields(s)
    jc = JumpConfig(K=a.K, relax=a.relax, m=a.m)
    if a.box:
        jc.box = tuple(int(v) for v in a.box.split("x"))
    from .perf import surrogate_source_hash
    out = {"workload": s.name, "steps": a.steps, "jump": jc.__dict__, "source_hash": surrogate_source_hash(),
           "runs": {}}
    if a.plain_from:
        out["runs"]["plain"] = json.load(open(a.plain_from))["runs"]["plain"]
        _log(f"[plain] reference trajectory from {a.plain_from}")
    else:
        sv = lbm.Solver(s.physics(), storage="f32")
        sv.init_fields(phi, u, ps)
        # statistics every plain_every steps, so that runs with other cycles find common steps
        out["runs"]["plain"] = run_plain(sv, a.steps, a.plain_every, log=_log)
        del sv
        torch.cuda.empty_cache()
    modes = a.modes.split(",")
    variants = [(mname, None, mname, {}) for mname in ("persistence", "transport", "comoving", "comoving_trend",
                                                       "projective")
                if mname in modes]
    if a.weights and ("network" in modes or "network_phi" in modes):
        net = Net(seed=0)
        load_weights(net, a.weights)
        if "network" in modes:
            variants.append(("surrogate", net, "network", {}))
        if "network_phi" in modes:         # the network's phase-field residual only
            variants.append(("surrogate_phi", net, "network", {"net_phi_only": True}))
    jc.predict_pressure = bool(a.predict_pressure)
    jc.velocity = a.velocity
    jc.max_gain = a.max_gain
    jc.accel_smooth = a.accel_smooth
    jc.warmup = a.warmup
    jc.accel = not a.no_accel
    jc.keep_neq = bool(a.keep_neq)
    jc.whole_cells = bool(a.whole_cells)
    jc.trend_gain = a.trend_gain
    jc.trend_bulk = bool(a.trend_bulk)
    jc.net_phi_only = bool(a.net_phi_only)
    jc.clip_phi = not a.no_clip
    jc.phi_at_interface = not a.no_phi_at_interface
    for name, net, mode, over in variants:
        sv = lbm.Solver(s.physics(), storage="f32")
        sv.init_fields(phi, u, ps)
        r = run_with_jumps(net, sv, s, a.steps, dataclasses.replace(jc, **over), log=_log, mode=mode)
        r["errors"] = compare_trajectories(out["runs"]["plain"], r)
        r["speedup"] = out["runs"]["plain"]["seconds"] / r["seconds"]
        out["runs"][name] = r
        _log(f"[jump] {name}: speedup {r['speedup']:.2f}x, errors {r['errors']}")
        del sv
        torch.cuda.empty_cache()
    return out


def _cmd_convbench(a):
    """Times the network's convolutions on one batch of the training crop
    shape with HIP events on the current stream: each layer's forward
    convolution, input gradient and weight gradient alone (mean of a.reps
    launches after one warm-up), then the whole forward pass and the whole
    forward + backward pass.  FLOP counts are the algorithmic 2 x 27 x
    c_in x c_out per output voxel."""
    import torch
    n, dd, hh, ww = (int(v) for v in a.shape.split("x"))
    net = Net(seed=0)
    dev = net.device
    g = torch.Generator(device="cpu").manual_seed(1)
    x = (torch.randn((n, dd, hh, ww, 16), generator=g) * 0.5).to(dev, torch.bfloat16)
    stream = torch.cuda.current_stream(dev)
    levels = {"enc0": 1, "enc1": 2, "enc2": 4, "bot_": 8, "dec2": 4, "dec1": 2, "dec0": 1, "out": 1}

    def timed(fn, reps):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    layers = []
    for name, ci, co, act in LAYERS:
        f = levels[name[:4] if name != "out" else "out"]
        shp = (n, dd // f, hh // f, ww // f)
        V = shp[0] * shp[1] * shp[2] * shp[3]
        xi = (torch.randn(shp + (ci,), generator=g) * 0.5).to(dev, torch.bfloat16)
        dy = (torch.randn(shp + (co,), generator=g) * 0.5).to(dev, torch.bfloat16)
        d = net.p[name]
        y = torch.empty(shp + (co,), device=dev, dtype=torch.bfloat16)
        dx = torch.empty(shp + (ci,), device=dev, dtype=torch.bfloat16)
        ws = net._ws_for(xi, co)
        flop = 2.0 * 27 * ci * co * V
        t_f = timed(lambda: sg.sg_conv3d_fwd(xi, d["wt"], d["b"], co, co, act, SLOPE, y, 0), a.reps)
        t_d = (timed(lambda: sg.sg_conv3d_bwd_data(dy, d["wt"], dx, d["wm"]), a.reps)
               if ci % 32 == 0 else None)
        t_w = timed(lambda: sg.sg_conv3d_bwd_weight(xi, dy, d["gw"], d["gb"], ws), a.reps)
        rec = {"layer": name, "shape": list(shp), "c_in": ci, "c_out": co, "gflop": flop / 1e9,
               "fwd_ms": t_f, "fwd_tflops": flop / (t_f * 1e-3) / 1e12,
               "bwd_data_ms": t_d, "bwd_data_tflops": None if t_d is None else flop / (t_d * 1e-3) / 1e12,
               "bwd_weight_ms": t_w, "bwd_weight_tflops": flop / (t_w * 1e-3) / 1e12}
        layers.append(rec)
        bd = "-" if t_d is None else f"{t_d:.3f} ms {rec['bwd_data_tflops']:.0f} TF/s"
        _log(f"[convbench] {name:6s} {ci:3d}->{co:3d} {shp}: fwd {t_f:.3f} ms {rec['fwd_tflops']:.0f} TF/s, "
             f"bwd-data {bd}, bwd-weight {t_w:.3f} ms {rec['bwd_weight_tflops']:.0f} TF/s")
        del xi, dy, y, dx
    V0 = n * dd * hh * ww
    flop_fwd = flops_per_voxel() * V0
    t_net = timed(lambda: net.forward(x, keep=False), a.reps)

    def fwd_bwd():
        out = net.forward(x, keep=True)
        net.backward(torch.zeros(out.shape, device=dev, dtype=torch.bfloat16))

    t_fb = timed(fwd_bwd, max(1, a.reps // 2))
    res = {"shape": [n, dd, hh, ww], "layers": layers, "forward_ms": t_net,
           "forward_tflops": flop_fwd / (t_net * 1e-3) / 1e12, "forward_backward_ms": t_fb,
           "forward_backward_tflops": 3 * flop_fwd / (t_fb * 1e-3) / 1e12,
           "peak_tflops_bf16_dense": 2500.0}
    _log(f"[convbench] network forward {t_net:.2f} ms ({res['forward_tflops']:.0f} TF/s), forward+backward "
         f"{t_fb:.2f} ms ({res['forward_backward_tflops']:.0f} TF/s, counting 3x the forward FLOP)")
    return res


def _log(msg):
    import sys
    print(msg, file=sys.stderr, flush=True)


def main():
    import argparse
    ap = argparse.ArgumentParser(description="surrogate training data, training and jump study")
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--runs", type=int, default=200)
    t.add_argument("--lbm-steps", type=int, default=6000)
    t.add_argument("--pairs-per-run", type=int, default=10)
    t.add_argument("--train-steps", type=int, default=2000)
    t.add_argument("--batch", type=int, default=8)
    t.add_argument("--lr", type=float, default=2e-4)
    t.add_argument("--seed", type=int, default=0)
    t.add_argument("--m", type=int, default=25, help="steps between the trend states (<= 400)")
    t.add_argument("--K", type=int, default=200, help="steps the network jumps (a multiple of 50)")
    t.add_argument("--base", default="comoving", choices=["comoving", "comoving_trend", "transport"],
                   help="baseline whose residual the network learns")
    t.add_argument("--whole-cells", action="store_true",
                   help="co-moving baseline displaced by whole cells (the driver's --whole-cells)")
    t.add_argument("--rollout", action="store_true",
                   help="training states from the jump driver (co-moving trend jumps), targets K plain steps on")
    t.add_argument("--relax", type=int, default=250, help="relaxation steps per cycle of the rollout runs")
    t.add_argument("--cycles", type=int, default=20, help="jump cycles per rollout run")
    t.add_argument("--box", default=None, help="window bx x by x bz of the rollout samples")
    t.add_argument("--weights", default=None)
    t.add_argument("--out", default=None)
    j = sub.add_parser("jump")
    j.add_argument("--weights", default=None)
    j.add_argument("--steps", type=int, default=40000)
    j.add_argument("--K", type=int, default=200)
    j.add_argument("--relax", type=int, default=50)
    j.add_argument("--m", type=int, default=25, help="trend window (<= relax, or K + relax for cycle ends)")
    j.add_argument("--modes", default="persistence,transport,comoving,network",
                   help="jumps to run after the plain run: persistence, transport, comoving, comoving_trend, "
                        "projective, network, network_phi (the network's phase-field residual only)")
    j.add_argument("--grid", default=None, help="override the grid, e.g. 128x512x128")
    j.add_argument("--D", type=float, default=None, help="bubble diameter with --grid")
    j.add_argument("--eo", type=float, default=10.0, help="Eotvos number with --grid")
    j.add_argument("--box", default=None, help="prediction window bx x by x bz, e.g. 80x96x80")
    j.add_argument("--predict-pressure", action="store_true")
    j.add_argument("--plain-from", default=None, help="reuse the plain run of an earlier study (same setup)")
    j.add_argument("--no-phi-at-interface", action="store_true")
    j.add_argument("--plain-every", type=int, default=25, help="statistics cadence of the plain run")
    j.add_argument("--velocity", default="gas", choices=["gas", "centroid"], help="co-moving jump velocity")
    j.add_argument("--max-gain", type=float, default=0.02, help="co-moving velocity factor limit")
    j.add_argument("--warmup", type=int, default=0, help="plain LBM steps before the first jump")
    j.add_argument("--accel-smooth", type=float, default=1.0,
                   help="weight of the newest acceleration estimate in its running average")
    j.add_argument("--no-accel", action="store_true", help="co-moving jumps without the trend window")
    j.add_argument("--no-clip", action="store_true", help="do not clip the jumped phi to [phi_L, phi_H]")
    j.add_argument("--keep-neq", action="store_true",
                   help="keep the populations' non-equilibrium parts after a jump (default: rebuild at equilibrium)")
    j.add_argument("--trend-gain", type=float, default=1.0, help="co-moving trend jump: factor on K/m")
    j.add_argument("--net-phi-only", action="store_true",
                   help="apply only the network's phase-field residual; the velocity follows the baseline")
    j.add_argument("--trend-bulk", action="store_true",
                   help="co-moving trend jump: velocity trend in the bulk of the heavy phase only")
    j.add_argument("--whole-cells", action="store_true",
                   help="co-moving displacement rounded to whole cells, the remainder carried to the next jump")
    j.add_argument("--out", default=None)
    c = sub.add_parser("convbench")
    c.add_argument("--shape", default="8x64x96x64", help="batch x D x H x W of the network input")
    c.add_argument("--reps", type=int, default=10)
    c.add_argument("--out", default=None)
    a = ap.parse_args()
    res = {"train": _cmd_train, "jump": _cmd_jump, "convbench": _cmd_convbench}[a.cmd](a)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
