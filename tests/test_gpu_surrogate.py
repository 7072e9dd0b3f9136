"""GPU parity of the surrogate-network kernels (through the sg_* C ABI)
against the FP64 CPU oracle on the same BF16-rounded operands.

Bar per element: |gpu - oracle| <= half a BF16 ulp of the stored result (when
the result is stored as BF16) + gamma_K * sum |terms|, gamma_K = K eps32 for
an FP32 accumulation of K products (K = 27 c_in for the forward and input
gradient, the voxel count for the weight gradient).
"""
import numpy as np
import pytest

from oracle import conv as oc

pytestmark = pytest.mark.gpu

EPS32 = float(np.finfo(np.float32).eps)


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_2012_06144_amd import sg
    return torch, sg


def _bf16(torch, a):
    t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda").to(torch.bfloat16)
    return t, t.float().cpu().numpy().astype(np.float64)


def _ulp_bf16(v):
    e = np.floor(np.log2(np.maximum(np.abs(v), 2.0 ** -126)))
    return 2.0 ** (e - 7)


CONV_CASES = [
    # (n, d, h, w, ci, co, n_store, act, f32_out)
    (1, 4, 6, 8, 16, 32, 32, 1, 0),       # first-layer width, partial block of voxels
    (2, 3, 5, 7, 32, 64, 64, 1, 0),       # ragged voxel count
    (1, 4, 4, 4, 48, 96, 96, 0, 0),       # three column tiles
    (1, 2, 4, 8, 64, 256, 256, 1, 0),     # two column groups of four tiles
    (1, 4, 4, 8, 32, 32, 5, 0, 1),        # FP32 output, first 5 channels kept
    # boxes of 32-wide rows (W > 16): partial in every direction, two boxes along W
    (1, 5, 7, 20, 32, 64, 64, 1, 0),
    (1, 3, 3, 40, 32, 32, 32, 1, 0),
    # boxes of 16-wide row pairs (8 < W <= 16), two samples
    (2, 6, 9, 13, 16, 64, 64, 0, 0),
]


@pytest.mark.parametrize("case", CONV_CASES)
def test_conv3d_fwd(env, case):
    torch, sg = env
    n, d, h, w, ci, co, ns, act, f32 = case
    rng = np.random.default_rng(hash(case) % 2 ** 32)
    xt, x = _bf16(torch, rng.standard_normal((n, d, h, w, ci)))
    wt, wv = _bf16(torch, rng.standard_normal((27, co, ci)) / np.sqrt(27 * ci))
    b = rng.standard_normal(co).astype(np.float32)
    bt = torch.from_numpy(b).cuda()
    y = torch.empty((n, d, h, w, ns), device="cuda", dtype=torch.float32 if f32 else torch.bfloat16)
    sg.sg_conv3d_fwd(xt, wt, bt, co, ns, act, 0.1, y, f32)
    torch.cuda.synchronize()
    ref = oc.conv3d(x, wv, b.astype(np.float64))
    if act:
        ref = oc.leaky(ref, 0.1)
    ref = ref[..., :ns]
    mag = oc.conv3d(np.abs(x), np.abs(wv), np.abs(b.astype(np.float64)))[..., :ns]
    bound = 27 * ci * EPS32 * mag + (0.0 if f32 else 1.0) * 0.5 * _ulp_bf16(ref) + 1e-30
    got = y.float().cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - ref) <= bound), np.max(np.abs(got - ref) / bound)


@pytest.mark.parametrize("case", [(1, 4, 6, 8, 32, 64), (2, 3, 5, 7, 64, 32), (1, 2, 4, 8, 96, 192),
                                  (1, 3, 5, 24, 32, 64)])
def test_conv3d_input_gradient(env, case):
    torch, sg = env
    n, d, h, w, ci, co = case
    rng = np.random.default_rng(sum(case))
    dyt, dy = _bf16(torch, rng.standard_normal((n, d, h, w, co)))
    wt, wv = _bf16(torch, rng.standard_normal((27, co, ci)) / np.sqrt(27 * co))
    wm = torch.empty((27, ci, co), device="cuda", dtype=torch.bfloat16)
    dx = torch.empty((n, d, h, w, ci), device="cuda", dtype=torch.bfloat16)
    sg.sg_conv3d_bwd_data(dyt, wt, dx, wm)
    torch.cuda.synchronize()
    # the workspace holds the mirrored weights wm[26 - t][ci][co] = wt[t][co][ci]
    assert torch.equal(wm, wt.flip(0).transpose(1, 2).contiguous())
    ref = oc.conv3d_bwd_data(dy, wv)
    mag = oc.conv3d_bwd_data(np.abs(dy), np.abs(wv))
    bound = 27 * co * EPS32 * mag + 0.5 * _ulp_bf16(ref) + 1e-30
    got = dx.float().cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - ref) <= bound), np.max(np.abs(got - ref) / bound)


@pytest.mark.parametrize("case", [
    (1, 4, 6, 8, 16, 32), (2, 5, 6, 7, 32, 64), (1, 4, 4, 4, 96, 32),
    # W rows padded to whole 16-voxel steps (W = 40 -> 48, W = 21 -> 32),
    # many (co, ci) tiles (8 x 4), wall-to-wall zero padding in d and h
    (1, 4, 8, 40, 128, 256), (1, 5, 13, 21, 128, 256),
    # more K steps (2025) than the plan's chunks: 2 steps per chunk, empty
    # chunks up to a multiple of 8, the two-level chunk sum (32 groups)
    (3, 15, 15, 40, 32, 32),
    # 5 steps per chunk with H = 4: a chunk's h runs end inside it and restart
    # on the next (n, d) plane or 16-voxel column, as in the full-size layers
    # (W = 200 -> 208, 13 columns, 4992 steps in 1000 chunks)
    (2, 48, 4, 200, 32, 32),
])
def test_conv3d_weight_gradient(env, case):
    torch, sg = env
    n, d, h, w, ci, co = case
    rng = np.random.default_rng(3 * sum(case))
    xt, x = _bf16(torch, rng.standard_normal((n, d, h, w, ci)))
    dyt, dy = _bf16(torch, rng.standard_normal((n, d, h, w, co)))
    dw = torch.empty((27, co, ci), device="cuda", dtype=torch.float32)
    db = torch.empty(co, device="cuda", dtype=torch.float32)
    ws = torch.empty(sg.sg_bwd_weight_workspace(n, d, h, w, ci, co) // 4 + 1, device="cuda", dtype=torch.float32)
    sg.sg_conv3d_bwd_weight(xt, dyt, dw, db, ws)
    torch.cuda.synchronize()
    rw, rb = oc.conv3d_bwd_weight(x, dy)
    mw, mb = oc.conv3d_bwd_weight(np.abs(x), np.abs(dy))
    V = n * d * h * w
    assert np.all(np.abs(dw.cpu().numpy() - rw) <= V * EPS32 * mw + 1e-30)
    assert np.all(np.abs(db.cpu().numpy() - rb) <= V * EPS32 * mb + 1e-30)


def test_resampling_and_elementwise(env):
    torch, sg = env
    rng = np.random.default_rng(11)
    xt, x = _bf16(torch, rng.standard_normal((2, 4, 6, 8, 16)))
    p = torch.empty((2, 2, 3, 4, 16), device="cuda", dtype=torch.bfloat16)
    sg.sg_pool2_fwd(xt, p)
    ref = oc.pool2(x)
    assert np.all(np.abs(p.float().cpu().numpy() - ref) <= 0.5 * _ulp_bf16(ref) + 8 * EPS32 * np.abs(ref))
    u = torch.empty_like(xt)
    sg.sg_up2_fwd(p, u)
    assert np.array_equal(u.float().cpu().numpy(), oc.up2(p.float().cpu().numpy().astype(np.float64)))
    dp = torch.empty_like(p)
    sg.sg_up2_bwd(xt, dp)
    ref_u = 8 * oc.pool2(x)
    assert np.all(np.abs(dp.float().cpu().numpy() - ref_u) <= 0.5 * _ulp_bf16(ref_u) + 8 * EPS32 * np.abs(ref_u) * 8)
    dx = torch.empty_like(xt)
    sg.sg_pool2_bwd(p, dx)
    ref_p = oc.up2(p.float().cpu().numpy().astype(np.float64)) / 8.0
    assert np.array_equal(dx.float().cpu().numpy().astype(np.float64), ref_p)
    a_t, a = _bf16(torch, rng.standard_normal((3, 5, 32)))
    b_t, b = _bf16(torch, rng.standard_normal((3, 5, 64)))
    cat = torch.empty((3, 5, 96), device="cuda", dtype=torch.bfloat16)
    sg.sg_concat(a_t, b_t, cat)
    assert np.array_equal(cat.float().cpu().numpy(), np.concatenate([a, b], -1))
    a2, b2 = torch.empty_like(a_t), torch.empty_like(b_t)
    sg.sg_split(cat, 32, 64, a2, b2)
    assert torch.equal(a2, a_t) and torch.equal(b2, b_t)
    s = torch.empty_like(a_t)
    sg.sg_add(a_t, a_t, s)
    assert np.array_equal(s.float().cpu().numpy(), 2 * a)
    yt, y = _bf16(torch, rng.standard_normal((1000,)))
    gt, g = _bf16(torch, rng.standard_normal((1000,)))
    d = torch.empty_like(yt)
    sg.sg_leaky_bwd(yt, gt, d, 0.1)
    ref_l = np.where(y > 0, g, 0.1 * g)
    assert np.all(np.abs(d.float().cpu().numpy() - ref_l) <= 0.5 * _ulp_bf16(ref_l))


def test_mse_and_adam(env):
    torch, sg = env
    rng = np.random.default_rng(12)
    p = rng.standard_normal(100000).astype(np.float32)
    t = rng.standard_normal(100000).astype(np.float32)
    loss = torch.zeros(1, device="cuda")
    scratch = torch.zeros(1024, device="cuda")
    g = torch.empty(100000, device="cuda", dtype=torch.bfloat16)
    sg.sg_mse(torch.from_numpy(p).cuda(), torch.from_numpy(t).cuda(), loss, g, scratch)
    torch.cuda.synchronize()
    rv, rg = oc.mse(p.astype(np.float64), t.astype(np.float64))
    assert abs(loss.item() - rv) <= 1e-5 * rv
    assert np.all(np.abs(g.float().cpu().numpy() - rg) <= 0.5 * _ulp_bf16(rg) + 4 * EPS32 * np.abs(rg))
    # Adam: 5 steps from the same state, FP32 vs FP64
    w0 = rng.standard_normal(5000)
    grads = [rng.standard_normal(5000) for _ in range(5)]
    pw, m, v = w0.copy(), np.zeros(5000), np.zeros(5000)
    tp = torch.from_numpy(w0.astype(np.float32)).cuda()
    tm = torch.zeros_like(tp)
    tv = torch.zeros_like(tp)
    tb = torch.empty(5000, device="cuda", dtype=torch.bfloat16)
    for k, gr in enumerate(grads, 1):
        oc.adam(pw, gr, m, v, 1e-2, 0.9, 0.999, 1e-8, k)
        sg.sg_adam(tp, torch.from_numpy(gr.astype(np.float32)).cuda(), tm, tv, tb, 1e-2, 0.9, 0.999, 1e-8, k)
    torch.cuda.synchronize()
    assert np.abs(tp.cpu().numpy() - pw).max() < 1e-5
    assert torch.equal(tb, tp.to(torch.bfloat16))


def test_field_packing_and_mass_projection(env):
    torch, sg = env
    rng = np.random.default_rng(13)
    nx, ny, nz = 12, 10, 8
    N = nx * ny * nz
    phi = rng.uniform(0, 1, N).astype(np.float32)
    u = rng.standard_normal(3 * N).astype(np.float32) * 1e-3
    p = rng.standard_normal(N).astype(np.float32) * 1e-4
    tphi, tu, tp = (torch.from_numpy(a).cuda() for a in (phi, u, p))
    box = (10, 2, 6, 8, 6, 4)          # wraps in x and z
    V = 8 * 6 * 4
    x = torch.empty((1, 4, 6, 8, 16), device="cuda", dtype=torch.bfloat16)
    st = torch.empty(V * 5, device="cuda", dtype=torch.float32)
    scale = [1.0, 1e-2, 1e-2, 1e-2, 1e-4]
    sg.sg_fields_to_input(tphi, tu, tp, nx, ny, nz, box, scale, 16, x, st)
    torch.cuda.synchronize()
    F = np.stack([phi, u[:N], u[N:2 * N], u[2 * N:], p], -1).reshape(nz, ny, nx, 5)
    zi = (6 + np.arange(4)) % nz
    yi = 2 + np.arange(6)
    xi = (10 + np.arange(8)) % nx
    ref = F[zi][:, yi][:, :, xi]
    assert np.array_equal(st.cpu().numpy().reshape(4, 6, 8, 5), ref)
    xs = x.float().cpu().numpy()
    assert np.all(xs[..., 5:] == 0)
    assert np.allclose(xs[..., :5], ref / np.array(scale), rtol=2 ** -8)
    # prediction applied back (walls at y = 0, ny-1 are skipped), phi clipped
    out = torch.from_numpy(rng.standard_normal((V, 32)).astype(np.float32)).cuda()
    so = [0.5, 1e-3, 1e-3, 1e-3, 1e-5]
    sg.sg_apply_prediction(out, 32, so, tphi, tu, tp, nx, ny, nz, box, 1, 0.0, 1.0)
    torch.cuda.synchronize()
    phi2 = tphi.cpu().numpy().reshape(nz, ny, nx)
    o = out.cpu().numpy().reshape(4, 6, 8, 32)
    expect = np.clip(ref[..., 0] + o[..., 0] * 0.5, 0, 1)
    assert np.allclose(phi2[zi][:, yi][:, :, xi], expect, atol=1e-6)


def _ulp32(v):
    e = np.floor(np.log2(np.maximum(np.abs(v), 2.0 ** -126)))
    return 2.0 ** (e - 23)


@pytest.mark.parametrize("walls,lo,hi", [(True, 0.0, 1.0), (True, 0.2, 1.4), (False, -1.0, 1.0)])
def test_mass_projection_matches_oracle(env, walls, lo, hi):
    """sg_mass_project against the FP64 oracle (orc_mass_project) per cell, on
    a grid with walls holding values no fluid cell has: each stored cell
    within one FP32 ulp of the oracle's value of the same FP32 input (the GPU
    rounds once; its FP64 sums differ by order only); wall rows and bulk
    cells bit-identical; the fluid sum at the target to the FP32 rounding of
    the stored cells."""
    torch, sg = env
    rng = np.random.default_rng(17)
    nz, ny, nx = 10, 13, 24
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r = np.sqrt((x - 11.3) ** 2 + (y - 6.2) ** 2 + (z - 4.9) ** 2)
    phi = lo + (hi - lo) * (0.5 + 0.5 * np.tanh(2 * (r - 3.5) / 3.0))
    phi += 1e-3 * rng.standard_normal(phi.shape) * (np.abs(r - 3.5) < 4)
    phi[:, :, 0] = lo                                  # exact bulk values
    phi[:, :, 1] = hi
    if walls:
        phi[:, 0, :] = 5.0
        phi[:, -1, :] = -5.0
    phi = phi.astype(np.float32).astype(np.float64)
    fluid = np.ones(phi.shape, dtype=bool)
    if walls:
        fluid[:, 0, :] = fluid[:, -1, :] = False
    target = float(phi[fluid].sum()) + 1.75
    pmin, pmax = min(lo, hi), max(lo, hi)
    ref = oc.mass_project(phi, walls, target, pmin, pmax)
    tphi = torch.from_numpy(phi.astype(np.float32)).cuda()
    scratch = torch.zeros(2048, device="cuda", dtype=torch.float64)
    sg.sg_mass_project(tphi, walls, target, pmin, pmax, scratch)
    torch.cuda.synchronize()
    got = tphi.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - ref) <= _ulp32(ref)), np.max(np.abs(got - ref) / _ulp32(ref))
    assert np.array_equal(got[~fluid], phi[~fluid])
    assert np.array_equal(got[:, 1:-1, :2], phi[:, 1:-1, :2])
    assert abs(got[fluid].sum() - target) <= 0.5 * _ulp32(got[fluid]).sum()


@pytest.mark.parametrize("case", [
    # (n, d, h, w, ca, cb, co): the decoder's three levels (64 + 32 -> 32 at W = 64 takes NT = 1, TW = 32;
    # 128 + 64 -> 64 at W = 32 NT = 2; 128 + 128 -> 128 at W = 16 NT = 1, TW = 16), a small-W case, and
    # partial boxes in d and h
    (2, 8, 6, 64, 64, 32, 32), (1, 4, 8, 32, 128, 64, 64), (2, 4, 6, 16, 128, 128, 128), (1, 6, 10, 8, 16, 48, 64),
])
def test_conv3d_fwd_up_cat_matches_the_formed_input(env, case):
    """sg_conv3d_fwd_up_cat(xa, xb) stages the same values as sg_conv3d_fwd
    on concat(up2(xa), xb) and runs the same products: bit-identical output,
    and the formed path is itself checked against the oracle (CONV_CASES)."""
    torch, sg = env
    n, d, h, w, ca, cb, co = case
    rng = np.random.default_rng(sum(case))
    xa, _ = _bf16(torch, rng.standard_normal((n, d // 2, h // 2, w // 2, ca)))
    xb, _ = _bf16(torch, rng.standard_normal((n, d, h, w, cb)))
    wt, _ = _bf16(torch, rng.standard_normal((27, co, ca + cb)) / np.sqrt(27 * (ca + cb)))
    bias = torch.from_numpy(rng.standard_normal(co).astype(np.float32)).cuda()
    up = torch.empty((n, d, h, w, ca), device="cuda", dtype=torch.bfloat16)
    sg.sg_up2_fwd(xa, up)
    cat = torch.empty((n, d, h, w, ca + cb), device="cuda", dtype=torch.bfloat16)
    sg.sg_concat(up, xb, cat)
    for act, f32 in ((1, 0), (0, 1)):
        dt = torch.float32 if f32 else torch.bfloat16
        y0 = torch.empty((n, d, h, w, co), device="cuda", dtype=dt)
        y1 = torch.full((n, d, h, w, co), float("nan"), device="cuda", dtype=dt)
        sg.sg_conv3d_fwd(cat, wt, bias, co, co, act, 0.1, y0, f32)
        sg.sg_conv3d_fwd_up_cat(xa, xb, wt, bias, co, co, act, 0.1, y1, f32)
        torch.cuda.synchronize()
        assert torch.equal(y0, y1), (case, act, f32)
    # an odd extent cannot be an upsampled one: refused before any launch
    status = sg._L.sg_conv3d_fwd_up_cat(sg._p(xa), ca, sg._p(xb), cb, n, d - 1, h, w, sg._p(wt), sg._p(bias), co,
                                        co, 1, 0.1, sg._p(y1), 0, None)
    assert status == -1 and b"even" in sg._L.sg_last_error()


def test_network_inference_forward_matches_training_forward(env):
    """Net.forward(keep=False) reads the decoder's [up2(coarse), skip] inputs
    directly; keep=True forms them for the backward pass: same output bits."""
    torch, sg = env
    from paper_2012_06144_amd import surrogate as S
    net = S.Net(seed=9)
    rng = np.random.default_rng(9)
    x, _ = _bf16(torch, rng.standard_normal((2, 16, 24, 16, S.C_IN)) * 0.5)
    a = net.forward(x, keep=True)
    b = net.forward(x, keep=False)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_network_gradient_against_oracle(env):
    """The whole encoder-decoder: loss gradient of the GPU network (BF16
    activations, FP32 accumulation) against the same network built from the
    oracle's FP64 operations on the same BF16-rounded weights and input.  BF16
    rounding of every activation limits agreement; the gradients must point
    the same way (cosine > 0.98) and agree in norm within 10 %."""
    torch, sg = env
    from paper_2012_06144_amd import surrogate as S
    net = S.Net(seed=5)
    rng = np.random.default_rng(14)
    xt, x = _bf16(torch, rng.standard_normal((1, 8, 8, 8, 16)) * np.r_[np.ones(5), np.zeros(11)])
    tgt = rng.standard_normal((1, 8, 8, 8, 32)).astype(np.float32)
    tgt[..., 5:] = 0
    out = net.forward(xt)
    loss = torch.zeros(1, device="cuda")
    scratch = torch.zeros(1024, device="cuda")
    g = torch.empty(out.shape, device="cuda", dtype=torch.bfloat16)
    sg.sg_mse(out, torch.from_numpy(tgt).cuda(), loss, g, scratch)
    net.backward(g)
    torch.cuda.synchronize()
    W = {k: d["wt"].float().cpu().numpy().astype(np.float64) for k, d in net.p.items()}
    B = {k: d["b"].cpu().numpy().astype(np.float64) for k, d in net.p.items()}

    def fwd(x):
        a = {}
        c = lambda k, t, act=True: oc.leaky(oc.conv3d(t, W[k], B[k]), 0.1) if act else oc.conv3d(t, W[k], B[k])
        a["x"] = x
        a["e0a"] = c("enc0a", x); a["s0"] = c("enc0b", a["e0a"]); a["p1"] = oc.pool2(a["s0"])
        a["e1a"] = c("enc1a", a["p1"]); a["s1"] = c("enc1b", a["e1a"]); a["p2"] = oc.pool2(a["s1"])
        a["e2a"] = c("enc2a", a["p2"]); a["s2"] = c("enc2b", a["e2a"]); a["p3"] = oc.pool2(a["s2"])
        a["ba"] = c("bot_a", a["p3"]); a["bb"] = c("bot_b", a["ba"])
        a["c2"] = np.concatenate([oc.up2(a["bb"]), a["s2"]], -1)
        a["d2a"] = c("dec2a", a["c2"]); a["t2"] = c("dec2b", a["d2a"])
        a["c1"] = np.concatenate([oc.up2(a["t2"]), a["s1"]], -1)
        a["d1a"] = c("dec1a", a["c1"]); a["t1"] = c("dec1b", a["d1a"])
        a["c0"] = np.concatenate([oc.up2(a["t1"]), a["s0"]], -1)
        a["d0a"] = c("dec0a", a["c0"]); a["t0"] = c("dec0b", a["d0a"])
        return c("out", a["t0"], act=False), a

    ref_out, a = fwd(x)
    _, gout = oc.mse(ref_out, tgt.astype(np.float64))
    # reverse pass with the oracle's operations
    G = {}

    def bw(k, xin, y, dy, act=True):
        dp = dy * np.where(y > 0, 1.0, 0.1) if act else dy
        G[k] = oc.conv3d_bwd_weight(xin, dp)[0]
        return oc.conv3d_bwd_data(dp, W[k])
    gt0 = bw("out", a["t0"], None, gout, act=False)
    g = bw("dec0b", a["d0a"], a["t0"], gt0); g = bw("dec0a", a["c0"], a["d0a"], g)
    gs0 = g[..., 64:]; g = oc.pool2(g[..., :64]) * 8
    g = bw("dec1b", a["d1a"], a["t1"], g); g = bw("dec1a", a["c1"], a["d1a"], g)
    gs1 = g[..., 128:]; g = oc.pool2(g[..., :128]) * 8
    g = bw("dec2b", a["d2a"], a["t2"], g); g = bw("dec2a", a["c2"], a["d2a"], g)
    gs2 = g[..., 128:]; g = oc.pool2(g[..., :128]) * 8
    g = bw("bot_b", a["ba"], a["bb"], g); g = bw("bot_a", a["p3"], a["ba"], g)
    gs2 = gs2 + oc.up2(g) / 8
    g = bw("enc2b", a["e2a"], a["s2"], gs2); g = bw("enc2a", a["p2"], a["e2a"], g)
    gs1 = gs1 + oc.up2(g) / 8
    g = bw("enc1b", a["e1a"], a["s1"], gs1); g = bw("enc1a", a["p1"], a["e1a"], g)
    gs0 = gs0 + oc.up2(g) / 8
    g = bw("enc0b", a["e0a"], a["s0"], gs0); bw("enc0a", a["x"], a["e0a"], g)
    for k in ("out", "dec0a", "dec2b", "bot_a", "enc1b", "enc0a"):
        gg = net.p[k]["gw"].cpu().numpy().ravel().astype(np.float64)
        rr = G[k].ravel()
        cos = gg @ rr / (np.linalg.norm(gg) * np.linalg.norm(rr))
        assert cos > 0.98, (k, cos)
        assert abs(np.linalg.norm(gg) / np.linalg.norm(rr) - 1) < 0.1, k


@pytest.fixture(scope="module")
def gain_data(env):
    from paper_2012_06144_amd import surrogate as S
    cfg = S.DataConfig(n_runs=4, grid=(64, 128, 64), d_range=(12.0, 16.0), eo_range=(5.0, 15.0), offset=4.0,
                       centre_y=40.0, steps=1400, start=200, every=50, K=200, pairs_per_run=6, box=(32, 48, 32))
    Sm, S0, S1, run_of, _ = S.generate_snapshots(cfg, log=lambda m: None)
    return cfg, Sm, S0, S1, run_of


@pytest.mark.parametrize("base", ["transport", "comoving"])
def test_trained_network_beats_the_method_without_it(env, gain_data, base):
    """What the learned part gains over the method without it: on held-out
    rising-bubble runs the jump of 200 steps with the trained network
    (baseline + learned residual, from the state and its recent trend) has
    a smaller error than its baseline alone, which in turn beats
    persistence (the state left as it is).  Baselines: phi transported by
    the local velocity, or the whole window translated with the bubble."""
    torch, sg = env
    from paper_2012_06144_amd import surrogate as S
    cfg, Sm, S0, S1, run_of = gain_data
    net = S.Net(seed=1)
    net.base = base
    shifts = S.comoving_shift(S0, S0.shape[0], cfg.box, cfg.K, prev=Sm, m=cfg.m) if base == "comoving" else None
    net.scale_in, net.scale_out, net.scale_trend = S.channel_scales(Sm, S0, S1, cfg.box, cfg.K, cfg.m,
                                                                    base_kind=base, shifts=shifts)
    res = S.train(net, Sm, S0, S1, cfg.box, cfg.K, cfg.m, run_of=run_of, steps=150, batch=8, lr=5e-4,
                  warmup=15, val_frac=0.25, log=print, shifts=shifts)
    print(f"validation loss: network {res['val_loss']:.4e}, {base} baseline alone {res['val_loss_baseline']:.4e}, "
          f"transport {res['val_loss_transport']:.4e}, persistence {res['val_loss_persistence']:.4e}")
    assert np.isfinite(res["val_loss"])
    assert res["val_loss_baseline"] < res["val_loss_persistence"]
    assert res["val_loss"] < 0.8 * res["val_loss_baseline"]


def test_advect_phase_matches_oracle(env):
    """Jump baseline on two boxes, FP32 on the GPU vs FP64 oracle.  FP32
    forms the departure point x - K u with an error of at most
    2 eps32 (max extent + K |u|) cells, which moves the interpolated value by
    at most that times the largest neighbour difference, plus 8 eps32 |phi|
    for the blend."""
    torch, sg = env
    rng = np.random.default_rng(21)
    n, bz, by, bx = 2, 9, 11, 13
    st = rng.standard_normal((n, bz, by, bx, 5)).astype(np.float32)
    st[..., 1:4] *= 0.01
    K = 200.0
    ts = torch.from_numpy(st).cuda()
    out = torch.empty_like(ts)
    sg.sg_advect_phase(ts, n, bx, by, bz, K, out)
    torch.cuda.synchronize()
    ref = conv_oracle_advect(st.astype(np.float64), K)
    got = out.cpu().numpy().astype(np.float64)
    assert np.array_equal(got[..., 1:], st[..., 1:].astype(np.float64))
    phi = st[..., 0].astype(np.float64)
    jump = max(np.abs(np.diff(phi, axis=a)).max() for a in (1, 2, 3))
    pos = 2 * EPS32 * (max(bx, by, bz) + K * np.abs(st[..., 1:4]).max())
    bound = pos * jump + 8 * EPS32 * np.abs(phi).max()
    assert np.abs(got[..., 0] - ref[..., 0]).max() <= bound


def conv_oracle_advect(st, K):
    return oc.advect_phase(st, K)


def test_shift_boxes_matches_oracle(env):
    """Co-moving baseline on three boxes with different displacements (one
    pushing departure points out of the box) and velocity factors, FP32 on
    the GPU vs the FP64 oracle: the departure point x - d carries at most
    2 eps32 (max extent + |d|) cells of error, moving the value by that
    times the largest neighbour difference, plus 8 eps32 |s| for the blend
    and the factor, all times the largest factor."""
    torch, sg = env
    rng = np.random.default_rng(26)
    n, bz, by, bx = 3, 9, 11, 13
    st = rng.standard_normal((n, bz, by, bx, 5)).astype(np.float32)
    d = np.array([[0.37, -1.61, 0.52, 1.0], [0.0, 0.41, 0.0, 1.37], [-3.2, 20.0, 2.75, 0.5]], dtype=np.float32)
    ts = torch.from_numpy(st).cuda()
    out = torch.empty_like(ts)
    sg.sg_shift_boxes(ts, n, bx, by, bz, torch.from_numpy(d).cuda(), out)
    torch.cuda.synchronize()
    ref = oc.shift_boxes(st.astype(np.float64), d.astype(np.float64))
    got = out.cpu().numpy().astype(np.float64)
    s64 = st.astype(np.float64)
    jump = max(np.abs(np.diff(s64, axis=a)).max() for a in (1, 2, 3))
    bound = (2 * EPS32 * (max(bx, by, bz) + np.abs(d[:, :3]).max()) * jump + 8 * EPS32 * np.abs(s64).max()) * 1.37
    assert np.abs(got - ref).max() <= bound
    # an in-place call is refused
    with pytest.raises(sg.SgError):
        sg.sg_shift_boxes(ts, n, bx, by, bz, torch.from_numpy(d).cuda(), ts)


def test_comoving_trend_base_matches_oracle(env):
    """The co-moving trend jump, T_dK[s + (K/m)(s - T_dm[s_m])] with phi
    carried, against the same three steps in the FP64 oracle (shift_boxes,
    projective_step with phi_step off, shift_boxes) at the displacements the
    jump computed.  Bound: each translation adds the shift test's bound for
    its input; the projective step multiplies the first one's error by K/m
    and adds 8 eps32 (|s| + (K/m)|s - T s_m|)."""
    torch, sg = env
    from paper_2012_06144_amd import surrogate as sgm
    rng = np.random.default_rng(31)
    bz, by, bx = 12, 16, 10
    z, y, x = np.meshgrid(np.arange(bz), np.arange(by), np.arange(bx), indexing="ij")
    r = np.sqrt((x - 4.6) ** 2 + (y - 7.3) ** 2 + (z - 5.8) ** 2)
    s0 = np.zeros((bz, by, bx, 5))
    s0[..., 0] = 0.5 + 0.5 * np.tanh((r - 3.0) / 1.5)            # gas bubble of radius 3
    s0[..., 2] = 0.01 + 0.002 * np.sin(0.3 * y) + 1e-3 * rng.standard_normal(r.shape)
    s0[..., 1] = 1e-3 * np.cos(0.4 * x)
    s0[..., 4] = 1e-4 * r
    sm = s0.copy()
    sm[..., 0] = 0.5 + 0.5 * np.tanh((np.sqrt((x - 4.6) ** 2 + (y - 6.1) ** 2 + (z - 5.8) ** 2) - 3.0) / 1.5)
    sm[..., 1:4] *= 0.97
    s0, sm = s0.astype(np.float32), sm.astype(np.float32)
    K, m = 100, 150
    t0, tm = torch.from_numpy(s0).cuda().view(-1), torch.from_numpy(sm).cuda().view(-1)
    out = torch.empty_like(t0)
    sgm.comoving_trend_base(t0, tm, (bx, by, bz), K, m, 0.0, 1.0, True, out)
    d_m, d_k = sgm.bubble_frame_shifts(t0, tm, (bx, by, bz), K, m)
    torch.cuda.synchronize()
    dm, dk = d_m.cpu().numpy().astype(np.float64), d_k.cpu().numpy().astype(np.float64)
    assert dm[1] > 0.5 and dk[1] > 0.5 and dm[3] == 1.0 and dk[3] == 1.0
    s64, m64 = s0.astype(np.float64)[None], sm.astype(np.float64)[None]
    moved = oc.shift_boxes(m64, dm[None])
    ext = oc.projective_step(s64, moved, K / m, 0.0, 1.0, u_by_phase=True, p_step=False, phi_step=False)
    ref = oc.shift_boxes(ext, dk[None])[0]
    got = out.cpu().numpy().astype(np.float64).reshape(ref.shape)

    def shift_bound(a, d):
        jump = max(np.abs(np.diff(a, axis=k)).max() for k in (1, 2, 3))
        return 2 * EPS32 * (max(bx, by, bz) + np.abs(d[:3]).max()) * jump + 8 * EPS32 * np.abs(a).max()

    ratio = K / m
    e1 = shift_bound(m64, dm)
    e2 = ratio * e1 + 8 * EPS32 * (np.abs(s64).max() + ratio * np.abs(s64 - moved).max())
    bound = e2 + shift_bound(ext, dk)
    assert np.abs(got - ref).max() <= bound
    # phi is only translated: equal to the translated phi of s0
    assert np.abs(got[..., 0] - oc.shift_boxes(s64, dk[None])[0][..., 0]).max() <= shift_bound(s64, dk)


def test_box_moments_matches_oracle(env):
    """FP64 sums of FP32 inputs: |error| <= V eps64 x (sum of |terms|) per
    entry (ordering only); phi spans beyond [0, 1] to exercise the clip."""
    torch, sg = env
    rng = np.random.default_rng(27)
    n, bz, by, bx = 3, 17, 19, 21
    st = rng.uniform(-0.1, 1.1, (n, bz, by, bx, 5)).astype(np.float32)
    st[..., 1:4] = rng.standard_normal((n, bz, by, bx, 3)) * 1e-3
    out = torch.zeros(n * 8, device="cuda", dtype=torch.float64)
    sg.sg_box_moments(torch.from_numpy(st).cuda(), n, bx, by, bz, 1.0, 0.0, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(n, 8)
    ref = oc.box_moments(st.astype(np.float64), 1.0, 0.0)
    V = bx * by * bz
    z, y, x = np.meshgrid(np.arange(bz), np.arange(by), np.arange(bx), indexing="ij")
    chi = np.clip(1.0 - st[..., 0].astype(np.float64), 0, 1)
    for k in range(n):
        c = chi[k]
        scale = np.array([c.sum(), (c * x).sum(), (c * y).sum(), (c * z).sum(),
                          np.abs(c * st[k, ..., 1]).sum(), np.abs(c * st[k, ..., 2]).sum(),
                          np.abs(c * st[k, ..., 3]).sum(), 0.0])
        assert np.all(np.abs(got[k] - ref[k]) <= 4 * V * np.finfo(np.float64).eps * scale)
    assert np.all(got[:, 7] == 0)


def test_channel_moments(env):
    torch, sg = env
    rng = np.random.default_rng(22)
    a = (rng.standard_normal((100003, 5)) * np.array([1, 1e-3, 2e-3, 1e-3, 1e-5])).astype(np.float32)
    out = torch.zeros(16, device="cuda", dtype=torch.float64)
    scratch = torch.zeros(512 * 16, device="cuda", dtype=torch.float64)
    sg.sg_channel_moments(torch.from_numpy(a).cuda(), a.shape[0], 5, out, scratch)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    a64 = a.astype(np.float64)
    eps = np.finfo(np.float64).eps * a.shape[0]
    assert np.all(np.abs(o[:5] - a64.sum(0)) <= eps * np.abs(a64).sum(0))
    assert np.all(np.abs(o[8:13] - (a64 ** 2).sum(0)) <= eps * (a64 ** 2).sum(0))
    assert np.all(o[5:8] == 0) and np.all(o[13:] == 0)


def test_apply_prediction_onto_a_base(env):
    torch, sg = env
    rng = np.random.default_rng(23)
    nx, ny, nz = 10, 8, 6
    N = nx * ny * nz
    phi = torch.from_numpy(rng.uniform(0, 1, N).astype(np.float32)).cuda()
    u = torch.from_numpy(rng.standard_normal(3 * N).astype(np.float32)).cuda()
    p = torch.from_numpy(rng.standard_normal(N).astype(np.float32)).cuda()
    box = (7, 1, 4, 8, 6, 4)
    V = 8 * 6 * 4
    base = rng.uniform(0, 1, (V, 5)).astype(np.float32)
    out = rng.standard_normal((V, 32)).astype(np.float32)
    so = [0.1, 0.2, 0.3, 0.4, 0.0]
    p0 = p.clone()
    sg.sg_apply_prediction(torch.from_numpy(out).cuda(), 32, so, phi, u, p, nx, ny, nz, box, 0, 0.0, 1.0,
                           base=torch.from_numpy(base).cuda())
    torch.cuda.synchronize()
    zi, yi, xi = (4 + np.arange(4)) % nz, 1 + np.arange(6), (7 + np.arange(8)) % nx
    ph = phi.cpu().numpy().reshape(nz, ny, nx)[zi][:, yi][:, :, xi].reshape(-1)
    uu = u.cpu().numpy().reshape(3, nz, ny, nx)[:, zi][:, :, yi][:, :, :, xi].reshape(3, -1)
    f32 = np.float32
    assert np.array_equal(ph, np.clip(base[:, 0] + out[:, 0] * f32(0.1), 0, 1))
    for k in range(3):
        assert np.array_equal(uu[k], base[:, 1 + k] + out[:, 1 + k] * f32(so[1 + k]))
    pp = p.cpu().numpy().reshape(nz, ny, nx)[zi][:, yi][:, :, xi].reshape(-1)
    assert np.array_equal(pp, base[:, 4])            # zero scale: the base value
    # planes z = 2, 3 lie outside the box (z = 4, 5, 0, 1): unchanged
    assert torch.equal(p.view(nz, ny, nx)[2:4], p0.view(nz, ny, nx)[2:4])
    # without the clip phi keeps its over- and undershoots
    sg.sg_apply_prediction(torch.from_numpy(out).cuda(), 32, so, phi, u, p, nx, ny, nz, box, 0, 0.0, 1.0,
                           base=torch.from_numpy(base).cuda(), clip=False)
    torch.cuda.synchronize()
    ph = phi.cpu().numpy().reshape(nz, ny, nx)[zi][:, yi][:, :, xi].reshape(-1)
    raw = base[:, 0] + out[:, 0] * f32(0.1)
    assert (raw < 0).any() and (raw > 1).any()
    assert np.array_equal(ph, raw)


def test_apply_prediction_velocity_weighted_by_phase(env):
    torch, sg = env
    rng = np.random.default_rng(24)
    nx, ny, nz = 8, 6, 4
    N = nx * ny * nz
    phi = torch.zeros(N, device="cuda")
    u = torch.zeros(3 * N, device="cuda")
    p = torch.zeros(N, device="cuda")
    box = (0, 0, 0, nx, ny, nz)
    base = rng.uniform(-0.2, 1.2, (N, 5)).astype(np.float32)
    out = rng.standard_normal((N, 32)).astype(np.float32)
    so = [0.0, 1.0, 1.0, 1.0, 0.0]
    sg.sg_apply_prediction(torch.from_numpy(out).cuda(), 32, so, phi, u, p, nx, ny, nz, box, 0, 0.0, 1.0,
                           base=torch.from_numpy(base).cuda(), u_by_phase=True)
    torch.cuda.synchronize()
    w = np.clip(base[:, 0], 0, 1).astype(np.float32)
    uu = u.cpu().numpy().reshape(3, N)
    for k in range(3):
        assert np.array_equal(uu[k], base[:, 1 + k] + w * out[:, 1 + k])


@pytest.mark.parametrize("layout", ["planar", "last"])
def test_projective_step_matches_oracle(env, layout):
    """FP32 on the GPU vs the FP64 oracle on the same FP32 inputs: each
    output is s + ratio (s - s_prev) (times the heavy fraction for u), a
    handful of FP32 operations on O(1) values: |error| <= 8 eps32 (|s| +
    ratio |s - s_prev|)."""
    torch, sg = env
    rng = np.random.default_rng(25)
    n = 4099
    s = rng.uniform(-0.1, 1.1, (n, 5)).astype(np.float32)
    sp = (s + rng.uniform(-0.02, 0.02, (n, 5))).astype(np.float32)
    ratio = 8.0
    if layout == "planar":
        a, b, cs, vs = np.ascontiguousarray(s.T), np.ascontiguousarray(sp.T), n, 1
    else:
        a, b, cs, vs = s, sp, 1, 5
    ta, tb = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    out = torch.empty_like(ta)
    bound = 8 * EPS32 * (np.abs(a) + ratio * np.abs(a.astype(np.float64) - b)) + 1e-30
    for ubp, phi_step in ((2, 1), (0, 0), (1, 0), (1, 1)):
        sg.sg_projective_step(ta, tb, n, cs, vs, ratio, 0.0, 1.0, ubp, phi_step, 1, out)
        torch.cuda.synchronize()
        ref = oc.projective_step(a.astype(np.float64), b.astype(np.float64), ratio, 0.0, 1.0, u_by_phase=ubp,
                                 p_step=True, layout=layout, phi_step=bool(phi_step))
        assert np.all(np.abs(out.cpu().numpy() - ref) <= bound), (ubp, phi_step)
    with pytest.raises(sg.SgError):
        sg.sg_projective_step(ta, tb, n, cs, vs, ratio, 0.0, 1.0, 3, 1, 1, out)
    # in place (the arguments of the last call above)
    sg.sg_projective_step(ta, tb, n, cs, vs, ratio, 0.0, 1.0, 1, 1, 1, ta)
    torch.cuda.synchronize()
    assert torch.equal(ta, out)


def test_pair_to_input(env):
    torch, sg = env
    rng = np.random.default_rng(26)
    V = 1000
    s = rng.standard_normal((V, 5)).astype(np.float32)
    sp = (s + 0.01 * rng.standard_normal((V, 5))).astype(np.float32)
    si = [1.0, 2.0, 3.0, 4.0, 5.0]
    ts = [10.0, 20.0, 30.0, 40.0, 50.0]
    x = torch.empty((V, 16), device="cuda", dtype=torch.bfloat16)
    sg.sg_pair_to_input(torch.from_numpy(s).cuda(), torch.from_numpy(sp).cuda(), si, ts, 16, x)
    torch.cuda.synchronize()
    got = x.float().cpu().numpy()
    r1 = s / np.array(si, np.float32)
    r2 = (s - sp) * np.array(ts, np.float32)
    ref = np.clip(np.concatenate([r1, r2, np.zeros((V, 6), np.float32)], 1), -16, 16)
    ref = torch.from_numpy(ref).to(torch.bfloat16).float()
    assert np.array_equal(got, ref.numpy())


def test_apply_prediction_phi_increment_at_interface(env):
    torch, sg = env
    rng = np.random.default_rng(27)
    nx, ny, nz = 8, 6, 4
    N = nx * ny * nz
    phi = torch.zeros(N, device="cuda")
    u = torch.zeros(3 * N, device="cuda")
    p = torch.zeros(N, device="cuda")
    base = rng.uniform(-0.1, 1.1, (N, 5)).astype(np.float32)
    base[:10, 0], base[10:20, 0] = 0.0, 1.0                    # bulk light and heavy phase
    out = (rng.standard_normal((N, 32)) * 0.1).astype(np.float32)
    so = [1.0, 0.0, 0.0, 0.0, 0.0]
    sg.sg_apply_prediction(torch.from_numpy(out).cuda(), 32, so, phi, u, p, nx, ny, nz, (0, 0, 0, nx, ny, nz), 0,
                           0.0, 1.0, base=torch.from_numpy(base).cuda(), phi_at_interface=True)
    torch.cuda.synchronize()
    q = np.clip(base[:, 0], 0, 1).astype(np.float32)
    w = np.float32(4) * q * (np.float32(1) - q)
    ref = np.clip(base[:, 0] + w * out[:, 0], 0, 1)
    got = phi.cpu().numpy()
    assert np.array_equal(got[:20], base[:20, 0])            # bulk phases unchanged
    assert np.allclose(got, ref, rtol=0, atol=2 * np.finfo(np.float32).eps)


def test_jump_driver_comoving_cycles(env):
    """Three cycles of the jump driver on a small rising bubble, started from
    the same developed state as a plain run: every cycle is either accepted
    or rolled back, the statistics stay finite, the phase-field mass is that
    of the plain run (the mass projection restores it after each jump), and
    the co-moving jump (window translated with the bubble, flow amplitude
    following its acceleration) ends closer to the plain run's rise than
    persistence (fields left as they are during each jump)."""
    torch, sg = env
    from paper_2012_06144_amd import inputs, lbm
    from paper_2012_06144_amd import surrogate as S
    D, Eo = 12.0, 10.0
    s = inputs.rising_bubble(48, 96, 48, D=D, center=(24.0, 30.0, 24.0), g=Eo * 1e-4 / (D * D))
    jc = S.JumpConfig(K=100, relax=40, m=20, box=(32, 48, 32))
    total = jc.m + 3 * (jc.K + jc.relax)
    sv = lbm.Solver(s.physics(), storage="f32")
    sv.init_fields(*inputs.build_fields(s))
    sv.step(800)
    start = sv.new_state_buffer()
    sv.save_state(start)
    y0 = sv.stats()["centroid"][1]
    sv.step(total)
    plain = sv.stats()
    rise_p = plain["centroid"][1] - y0
    res = {}
    for mode in ("persistence", "comoving"):
        sv.restore_state(start)
        r = S.run_with_jumps(None, sv, s, total, jc, log=print, mode=mode)
        st = sv.stats()
        assert r["accepted"] + r["rejected"] == 3
        for e in r["trajectory"]:
            assert all(np.isfinite(e[k]) for k in ("centroid_y", "rise_velocity", "mass", "xi_eff"))
        assert abs(st["mass"] - plain["mass"]) <= 1e-5 * abs(plain["mass"])
        res[mode] = st["centroid"][1] - y0
    print(f"rise over {total} steps: plain {rise_p:.4f}, persistence {res['persistence']:.4f}, "
          f"co-moving {res['comoving']:.4f} cells")
    assert rise_p > 0
    assert abs(res["comoving"] - rise_p) < 0.5 * abs(res["persistence"] - rise_p)
