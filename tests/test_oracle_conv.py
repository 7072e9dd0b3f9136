"""Pins of the surrogate-network oracle (FP64 CPU): each operation against a
library routine or a property that does not come from the oracle itself.

* 3x3x3 convolution = scipy.ndimage.correlate per (C_out, C_in) pair, zero
  padding, plus bias.
* Gradient with respect to the input: the adjoint identity
  <conv(x, w), y> = <x, bwd_data(y, w)>.
* Gradient with respect to the weights: <conv(x, dw), y> = <dw, bwd_weight(x, y)>
  (the convolution is linear in w), db = sum of y; and central finite
  differences of an MSE loss.
* Pooling = numpy block mean; upsampling = numpy repeat; pooling is the
  adjoint of upsampling divided by 8.
* Adam with a constant gradient moves every parameter by exactly
  lr * g / (|g| + eps) per step (bias correction makes m_hat = g, v_hat = g^2).
* Jump baseline (semi-Lagrangian transport of phi): identity at zero
  velocity, an exact shift for integer displacements, exact on linear fields
  (trilinear interpolation reproduces them), clamping at the box faces.
"""
import numpy as np
import pytest
from scipy import ndimage

from oracle import conv


def _rand(*shape, seed=0):
    return np.random.default_rng(seed).standard_normal(shape)


@pytest.mark.parametrize("shape,ci,co", [((1, 4, 5, 6), 3, 2), ((2, 3, 3, 3), 5, 4), ((1, 1, 2, 7), 2, 3)])
def test_conv3d_matches_scipy_correlate(shape, ci, co):
    x = _rand(*shape, ci, seed=1)
    w = _rand(27, co, ci, seed=2)
    b = _rand(co, seed=3)
    y = conv.conv3d(x, w, b)
    ref = np.zeros(shape + (co,))
    for n in range(shape[0]):
        for o in range(co):
            acc = np.full(shape[1:], b[o])
            for i in range(ci):
                k = w[:, o, i].reshape(3, 3, 3)   # k[a+1, b+1, c+1] = w[t]
                acc += ndimage.correlate(x[n, ..., i], k, mode="constant", cval=0.0)
            ref[n, ..., o] = acc
    assert np.abs(y - ref).max() < 1e-12


def test_bwd_data_is_adjoint_of_conv():
    x = _rand(2, 4, 5, 3, 6, seed=4)
    w = _rand(27, 7, 6, seed=5)
    y = _rand(2, 4, 5, 3, 7, seed=6)
    lhs = np.sum(conv.conv3d(x, w) * y)
    rhs = np.sum(x * conv.conv3d_bwd_data(y, w))
    assert abs(lhs - rhs) < 1e-12 * (abs(lhs) + 1)


def test_bwd_weight_is_gradient_of_bilinear_form():
    x = _rand(1, 5, 4, 6, 3, seed=7)
    y = _rand(1, 5, 4, 6, 4, seed=8)
    dw = _rand(27, 4, 3, seed=9)
    gw, gb = conv.conv3d_bwd_weight(x, y)
    lhs = np.sum(conv.conv3d(x, dw) * y)
    assert abs(lhs - np.sum(dw * gw)) < 1e-12 * (abs(lhs) + 1)
    assert np.abs(gb - y.sum(axis=(0, 1, 2, 3))).max() < 1e-12


def test_conv_gradients_by_finite_differences():
    """L = mse(leaky(conv(x, w, b)), t): central differences (h = 1e-6) of a
    few weights, biases and inputs against the chain rule built from the
    oracle's backward operations."""
    slope = 0.1
    x = _rand(1, 3, 4, 3, 2, seed=10)
    w = 0.5 * _rand(27, 3, 2, seed=11)
    b = 0.1 * _rand(3, seed=12)
    t = _rand(1, 3, 4, 3, 3, seed=13)

    def loss(x, w, b):
        return conv.mse(conv.leaky(conv.conv3d(x, w, b), slope), t, want_grad=False)[0]

    pre = conv.conv3d(x, w, b)
    y = conv.leaky(pre, slope)
    _, gy = conv.mse(y, t)
    gpre = gy * np.where(pre > 0, 1.0, slope)
    gw, gb = conv.conv3d_bwd_weight(x, gpre)
    gx = conv.conv3d_bwd_data(gpre, w)
    h = 1e-6
    rng = np.random.default_rng(14)
    for _ in range(6):
        idx = tuple(rng.integers(0, s) for s in w.shape)
        wp, wm = w.copy(), w.copy()
        wp[idx] += h
        wm[idx] -= h
        fd = (loss(x, wp, b) - loss(x, wm, b)) / (2 * h)
        assert abs(fd - gw[idx]) < 1e-6 * max(1.0, abs(fd))
    for k in range(3):
        bp, bm = b.copy(), b.copy()
        bp[k] += h
        bm[k] -= h
        fd = (loss(x, w, bp) - loss(x, w, bm)) / (2 * h)
        assert abs(fd - gb[k]) < 1e-6 * max(1.0, abs(fd))
    for _ in range(6):
        idx = tuple(rng.integers(0, s) for s in x.shape)
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (loss(xp, w, b) - loss(xm, w, b)) / (2 * h)
        assert abs(fd - gx[idx]) < 1e-6 * max(1.0, abs(fd))


def test_pool_and_upsample():
    x = _rand(2, 4, 6, 2, 3, seed=15)
    p = conv.pool2(x)
    ref = x.reshape(2, 2, 2, 3, 2, 1, 2, 3).mean(axis=(2, 4, 6))
    assert np.abs(p - ref).max() < 1e-15
    c = _rand(2, 2, 3, 1, 3, seed=16)
    u = conv.up2(c)
    ref_u = np.repeat(np.repeat(np.repeat(c, 2, axis=1), 2, axis=2), 2, axis=3)
    assert np.array_equal(u, ref_u)
    # <pool(x), c> = <x, up(c)> / 8
    assert abs(np.sum(p * c) - np.sum(x * u) / 8.0) < 1e-12


def test_leaky_and_mse():
    x = _rand(5, 7, seed=17)
    assert np.array_equal(conv.leaky(x, 0.1), np.where(x > 0, x, 0.1 * x))
    t = _rand(5, 7, seed=18)
    v, g = conv.mse(x, t)
    assert abs(v - np.mean((x - t) ** 2)) < 1e-15
    assert np.abs(g - 2 * (x - t) / x.size).max() < 1e-15


def test_adam_constant_gradient():
    rng = np.random.default_rng(19)
    p0 = rng.standard_normal(50)
    g = rng.standard_normal(50)
    p = p0.copy()
    m = np.zeros(50)
    v = np.zeros(50)
    lr, eps = 1e-3, 1e-8
    for t in range(1, 11):
        conv.adam(p, g, m, v, lr, 0.9, 0.999, eps, t)
        expect = p0 - t * lr * g / (np.abs(g) + eps)
        assert np.abs(p - expect).max() < 1e-12


def _box_state(bz, by, bx, seed=0):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((bz, by, bx, 5))


def test_advect_zero_velocity_is_identity():
    s = _box_state(5, 6, 7)
    s[..., 1:4] = 0.0
    assert np.array_equal(conv.advect_phase(s, 200.0), s)


def test_advect_integer_shift_moves_the_field():
    """A uniform velocity with K u = (1, -2, 1) cells moves phi by that many
    cells; voxels whose departure point lies inside the box match exactly."""
    s = _box_state(6, 7, 8, seed=1)
    K = 200.0
    s[..., 1], s[..., 2], s[..., 3] = 1.0 / K, -2.0 / K, 1.0 / K
    o = conv.advect_phase(s, K)
    phi = s[..., 0]
    # out[z, y, x] = phi[z - 1, y + 2, x - 1]
    assert np.array_equal(o[1:, :-2, 1:, 0], phi[:-1, 2:, :-1])
    assert np.array_equal(o[..., 1:], s[..., 1:])


def test_advect_reproduces_linear_fields():
    """Trilinear interpolation is exact for a linear field: with a uniform
    non-integer displacement every interior voxel gets a + b.(x - K u)."""
    bz, by, bx = 6, 7, 8
    z, y, x = np.meshgrid(np.arange(bz), np.arange(by), np.arange(bx), indexing="ij")
    a, b = 0.3, np.array([0.05, -0.02, 0.07])       # along x, y, z
    s = np.zeros((bz, by, bx, 5))
    s[..., 0] = a + b[0] * x + b[1] * y + b[2] * z
    d = np.array([0.37, -1.61, 0.52])                # K u in cells, along x, y, z
    K = 100.0
    s[..., 1:4] = d / K
    o = conv.advect_phase(s, K)
    exact = a + b[0] * (x - d[0]) + b[1] * (y - d[1]) + b[2] * (z - d[2])
    inside = (x - d[0] >= 0) & (x - d[0] <= bx - 1) & (y - d[1] >= 0) & (y - d[1] <= by - 1) & \
             (z - d[2] >= 0) & (z - d[2] <= bz - 1)
    assert inside.sum() > 100
    assert np.max(np.abs(o[..., 0] - exact)[inside]) < 1e-14


def test_advect_clamps_departure_to_the_box():
    s = _box_state(4, 4, 4, seed=2)
    s[..., 1:4] = 0.0
    s[..., 1] = 10.0                                  # departure far left of x = 0
    o = conv.advect_phase(s, 1.0)
    assert np.array_equal(o[..., 0], np.broadcast_to(s[:, :, :1, 0], (4, 4, 4)))


def test_shift_boxes_integer_shift_moves_every_channel():
    s = _box_state(6, 7, 8, seed=4)
    d = np.array([[1.0, -2.0, 1.0]])                 # along x, y, z
    o = conv.shift_boxes(s, d)
    # out[z, y, x, :] = s[z - 1, y + 2, x - 1, :]
    assert np.array_equal(o[1:, :-2, 1:, :], s[:-1, 2:, :-1, :])
    assert np.array_equal(conv.shift_boxes(s, np.zeros((1, 3))), s)
    # the velocity factor scales u only
    o2 = conv.shift_boxes(s, np.array([[1.0, -2.0, 1.0, 1.5]]))
    assert np.array_equal(o2[..., 0], o[..., 0]) and np.array_equal(o2[..., 4], o[..., 4])
    assert np.allclose(o2[..., 1:4], 1.5 * o[..., 1:4], rtol=1e-15, atol=0)


def test_shift_boxes_reproduces_linear_fields_per_box():
    """Two boxes with different non-integer displacements: every channel of
    a linear field is translated exactly wherever the departure point lies
    inside the box."""
    bz, by, bx = 6, 7, 8
    z, y, x = np.meshgrid(np.arange(bz), np.arange(by), np.arange(bx), indexing="ij")
    rng = np.random.default_rng(5)
    a, B = rng.standard_normal(5), rng.standard_normal((5, 3)) * 0.1
    s = np.stack([a[k] + B[k, 0] * x + B[k, 1] * y + B[k, 2] * z for k in range(5)], axis=-1)
    d = np.array([[0.37, -1.61, 0.52], [-0.8, 0.25, 1.3]])
    o = conv.shift_boxes(np.stack([s, s]), d)
    for n in range(2):
        dx, dy, dz = d[n]
        inside = (x - dx >= 0) & (x - dx <= bx - 1) & (y - dy >= 0) & (y - dy <= by - 1) & \
                 (z - dz >= 0) & (z - dz <= bz - 1)
        assert inside.sum() > 50
        for k in range(5):
            exact = a[k] + B[k, 0] * (x - dx) + B[k, 1] * (y - dy) + B[k, 2] * (z - dz)
            assert np.max(np.abs(o[n, ..., k] - exact)[inside]) < 1e-13


def _bubble_box(dims, c, R, xi, u=(0.0, 0.0, 0.0)):
    """Box state (bz, by, bx, 5) (dims = (bx, by, bz)) with a gas bubble
    (phi = 0 inside, 1 outside, tanh profile of width xi) centred at c
    (x, y, z) and uniform velocity u."""
    bx, by, bz = dims
    z, y, x = np.meshgrid(np.arange(bz), np.arange(by), np.arange(bx), indexing="ij")
    r = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
    s = np.zeros((bz, by, bx, 5))
    s[..., 0] = 0.5 + 0.5 * np.tanh(2.0 * (r - R) / xi)
    s[..., 1:4] = u
    return s


def test_box_moments_of_a_bubble():
    """A bubble centred on a grid point has its gas centroid there (mirror
    symmetry); its gas volume is that of the tanh profile,
    4/3 pi R^3 + 8 pi R (xi/2)^2 pi^2/24 (the profile is odd about r = R, so
    only the 2 R s part of r^2 = (R + s)^2 adds, with the integral of
    t (1 - tanh t) over t > 0 equal to pi^2/24); the gas-weighted velocity
    of a uniform flow is that flow; phi outside [phi_light, phi_heavy]
    counts as pure phase."""
    R, xi = 6.0, 3.0
    # box extents odd and the centre in the middle: each axis is mirror-symmetric
    s = _bubble_box((27, 23, 25), (13.0, 11.0, 12.0), R, xi, u=(1e-3, -2e-3, 5e-4))
    m = conv.box_moments(s, 1.0, 0.0)[0]
    vol = 4.0 / 3.0 * np.pi * R ** 3 + 8.0 * np.pi * R * (xi / 2) ** 2 * np.pi ** 2 / 24
    assert abs(m[0] - vol) < 2e-3 * vol
    assert np.allclose(m[1:4] / m[0], [13.0, 11.0, 12.0], atol=1e-12, rtol=0)
    assert np.allclose(m[4:7] / m[0], [1e-3, -2e-3, 5e-4], atol=1e-15, rtol=1e-13)
    assert m[7] == 0.0
    t = s.copy()
    t[..., 0] = np.where(t[..., 0] < 0.5, -0.3, 1.4)  # overshoots clip to chi = 1 / 0
    mt = conv.box_moments(t, 1.0, 0.0)[0]
    assert mt[0] == np.count_nonzero(s[..., 0] < 0.5)
    # phi_heavy < phi_light flips the indicator: chi counts the other phase
    mf = conv.box_moments(s, 0.0, 1.0)[0]
    assert abs(mf[0] + m[0] - 27 * 23 * 25) < 1e-9


def test_shift_moves_the_gas_centroid_by_the_displacement():
    """Linear interpolation keeps the first moment of a blob away from the
    box edges: the centroid of the shifted box moves by exactly d."""
    s = _bubble_box((32, 34, 30), (15.5, 17.0, 14.0), 5.0, 2.0)  # tails ~1e-10 at the box faces
    d = np.array([[0.3, 0.41, -0.27]])
    m0 = conv.box_moments(s, 1.0, 0.0)[0]
    m1 = conv.box_moments(conv.shift_boxes(s, d), 1.0, 0.0)[0]
    assert abs(m1[0] - m0[0]) < 1e-9 * m0[0]
    assert np.allclose(m1[1:4] / m1[0] - m0[1:4] / m0[0], d[0], atol=1e-6, rtol=0)  # tails at the faces: ~1e-8


def test_projective_step_exact_for_fields_linear_in_time():
    """s(t) = a + b t for every channel: the projective step from s(t - m)
    and s(t) lands exactly on s(t + K) (u unweighted, p stepped, phi inside
    its bounds)."""
    rng = np.random.default_rng(3)
    a = rng.uniform(0.3, 0.7, (7, 5))
    b = rng.uniform(-1e-4, 1e-4, (7, 5))
    t, m, K = 1000.0, 25.0, 200.0
    s_prev, s = a + b * (t - m), a + b * t
    out = conv.projective_step(s, s_prev, K / m, 0.0, 1.0, u_by_phase=False, p_step=True)
    assert np.max(np.abs(out - (a + b * (t + K)))) < 1e-15


def test_projective_step_limits():
    rng = np.random.default_rng(4)
    s = rng.uniform(0.0, 1.0, (50, 5))
    sp = s + rng.uniform(-0.1, 0.1, (50, 5))
    # ratio 0: identity
    assert np.array_equal(conv.projective_step(s, sp, 0.0, 0.0, 1.0), s)
    out = conv.projective_step(s, sp, 8.0, 0.0, 1.0, u_by_phase=True, p_step=False)
    # phi clipped into [0, 1]; pressure carried over
    assert out[:, 0].min() >= 0.0 and out[:, 0].max() <= 1.0
    assert np.array_equal(out[:, 4], s[:, 4])
    # velocity increments scale with the heavy-phase fraction: none in the
    # light phase (phi = 0), all of it in the heavy phase (phi = 1)
    s2 = s.copy()
    s2[:25, 0], s2[25:, 0] = 0.0, 1.0
    out2 = conv.projective_step(s2, sp, 8.0, 0.0, 1.0, u_by_phase=True)
    assert np.array_equal(out2[:25, 1:4], s2[:25, 1:4])
    assert np.allclose(out2[25:, 1:4], s2[25:, 1:4] + 8.0 * (s2[25:, 1:4] - sp[25:, 1:4]), rtol=0, atol=1e-15)
    # u_by_phase = 2: the bulk of the heavy phase only (weight clamp(10 q - 9, 0, 1))
    s4 = s2.copy()
    s4[:, 0] = np.linspace(0.0, 1.0, 50)
    out4 = conv.projective_step(s4, sp, 8.0, 0.0, 1.0, u_by_phase=2)
    w = np.clip(10.0 * s4[:, 0] - 9.0, 0.0, 1.0)
    assert np.allclose(out4[:, 1:4], s4[:, 1:4] + w[:, None] * 8.0 * (s4[:, 1:4] - sp[:, 1:4]), rtol=0, atol=1e-15)
    assert np.array_equal(out4[s4[:, 0] <= 0.9, 1:4], s4[s4[:, 0] <= 0.9, 1:4])
    # phi_step off: phi carried over (clipped), the other channels stepped as before
    s3 = s2.copy()
    s3[:5, 0] = 1.2
    out3 = conv.projective_step(s3, sp, 8.0, 0.0, 1.0, u_by_phase=True, phi_step=False)
    assert np.array_equal(out3[:, 0], np.clip(s3[:, 0], 0.0, 1.0))
    assert np.array_equal(out3[5:, 1:], conv.projective_step(s3, sp, 8.0, 0.0, 1.0, u_by_phase=True)[5:, 1:])


def test_projective_step_layouts_agree():
    rng = np.random.default_rng(5)
    s = rng.uniform(0.0, 1.0, (3, 4, 6, 5))
    sp = s + rng.uniform(-0.01, 0.01, s.shape)
    last = conv.projective_step(s, sp, 8.0, 0.0, 1.0)
    planar = conv.projective_step(np.moveaxis(s, -1, 0), np.moveaxis(sp, -1, 0), 8.0, 0.0, 1.0, layout="planar")
    assert np.array_equal(np.moveaxis(planar, 0, -1), last)


def _tanh_field(nz, ny, nx, lo, hi, R=4.0, xi=3.0):
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r = np.sqrt((x - nx / 2 + 0.3) ** 2 + (y - ny / 2 - 0.2) ** 2 + (z - nz / 2 + 0.1) ** 2)
    return lo + (hi - lo) * (0.5 + 0.5 * np.tanh(2 * (r - R) / xi))


@pytest.mark.parametrize("lo,hi", [(0.0, 1.0), (0.2, 1.4), (1.0, -1.0)])
def test_mass_projection_hits_the_target_inside_the_interface(lo, hi):
    """Mass projection of the jump: the fluid-cell sum of the result equals the
    target to FP64 rounding; cells in either bulk phase (phi = phi_min or
    phi_max exactly), over- and undershooting cells, and wall rows are left
    unchanged; the correction is largest at the mid value and symmetric in q
    and 1 - q (a multiple of 4 q (1 - q)).  The third case has phi_H < phi_L."""
    nz, ny, nx = 9, 14, 11
    phi = _tanh_field(nz, ny, nx, lo, hi)
    pmin, pmax = min(lo, hi), max(lo, hi)
    phi[2, 5, 3], phi[2, 5, 4] = pmin, pmax                 # exact bulk values
    phi[3, 6, 2], phi[3, 6, 3] = pmin - 1e-3, pmax + 1e-3   # outside the interval
    phi[4, 7, 5], phi[4, 7, 6] = 0.5 * (lo + hi), lo + 0.25 * (hi - lo)
    phi[4, 7, 7] = lo + 0.75 * (hi - lo)
    phi[:, 0, :] = 7.0                                      # wall rows (a value no fluid cell has)
    phi[:, -1, :] = -7.0
    fluid = np.ones(phi.shape, dtype=bool)
    fluid[:, 0, :] = fluid[:, -1, :] = False
    target = phi[fluid].sum() + 2.5
    out = conv.mass_project(phi, True, target, pmin, pmax)
    assert abs(out[fluid].sum() - target) <= 64 * np.finfo(float).eps * np.abs(phi[fluid]).sum()
    for idx in ((2, 5, 3), (2, 5, 4), (3, 6, 2), (3, 6, 3)):
        assert out[idx] == phi[idx]
    assert np.array_equal(out[~fluid], phi[~fluid])
    d = out - phi
    mid, quarter, three = d[4, 7, 5], d[4, 7, 6], d[4, 7, 7]
    assert mid > 0 and abs(d[fluid]).max() <= mid * (1 + 1e-12)
    assert abs(quarter - three) <= 1e-12 * mid                 # q = 1/4 and 3/4 move alike
    assert abs(quarter / mid - 0.75) <= 1e-12                  # 4 q (1 - q) = 3/4 at q = 1/4
    # without walls every row takes part
    phi2 = _tanh_field(nz, ny, nx, lo, hi)
    out2 = conv.mass_project(phi2, False, phi2.sum() - 1.0, pmin, pmax)
    assert abs(out2.sum() - (phi2.sum() - 1.0)) <= 64 * np.finfo(float).eps * np.abs(phi2).sum()


def test_mass_projection_of_a_bulk_field_changes_nothing():
    """With no interface cell there is nothing to move: the field is returned
    unchanged whatever the target."""
    phi = np.ones((4, 5, 6))
    phi[:, :, :3] = 0.0
    out = conv.mass_project(phi, False, phi.sum() + 1.0, 0.0, 1.0)
    assert np.array_equal(out, phi)
