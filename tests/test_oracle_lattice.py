"""Pins of the oracle's local pieces against what the mathematics fixes.

Each test checks one ingredient of the oracle against a fact that does not
come from the oracle itself: isotropy conditions that determine the lattice
weights, moments of the equilibria, the forcing identities, the closed form
of the moment-space collision, and exactness of the finite-difference
stencils on polynomials.
"""
import itertools

import numpy as np
import pytest

from oracle import oracle as orc

CS2 = 1.0 / 3.0


def _iso_tensors(e, w):
    e = e.astype(np.float64)
    m0 = w.sum()
    m1 = np.einsum("i,ia->a", w, e)
    m2 = np.einsum("i,ia,ib->ab", w, e, e)
    m3 = np.einsum("i,ia,ib,ic->abc", w, e, e, e)
    m4 = np.einsum("i,ia,ib,ic,id->abcd", w, e, e, e, e)
    return m0, m1, m2, m3, m4


def _delta4():
    d = np.eye(3)
    return (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
            + np.einsum("ad,bc->abcd", d, d))


@pytest.mark.parametrize("q", [15, 19, 27])
def test_velocity_set_structure(q):
    """D3Q15 = rest + 6 axes + 8 corners; D3Q19 = rest + 6 axes + 12 edges;
    D3Q27 = all of {-1,0,1}^3; each odd index has its opposite at the next
    index (used by bounce-back)."""
    e, w = orc.velocity_set(q)
    vecs = {tuple(v) for v in e}
    assert len(vecs) == q
    if q == 27:
        assert vecs == set(itertools.product((-1, 0, 1), repeat=3))
    else:
        norms = sorted(int(np.abs(v).sum()) for v in e)
        assert norms == [0] + [1] * 6 + ([3] * 8 if q == 15 else [2] * 12)
    assert tuple(e[0]) == (0, 0, 0)
    for i in range(1, q, 2):
        assert np.array_equal(e[i + 1], -e[i])


@pytest.mark.parametrize("q", [15, 19, 27])
def test_weights_isotropy(q):
    """P1: sum w = 1, sum w e = 0, sum w e e = cs^2 I, sum w e e e = 0,
    sum w e e e e = cs^4 (dd + dd + dd)."""
    e, w = orc.velocity_set(q)
    m0, m1, m2, m3, m4 = _iso_tensors(e, w)
    assert abs(m0 - 1.0) < 1e-15
    assert np.abs(m1).max() < 1e-15
    assert np.abs(m2 - CS2 * np.eye(3)).max() < 1e-15
    assert np.abs(m3).max() < 1e-15
    assert np.abs(m4 - CS2 * CS2 * _delta4()).max() < 1e-15


@pytest.mark.parametrize("q", [15, 19, 27])
def test_weights_are_the_unique_isotropic_solution(q):
    """The class weights solve the isotropy conditions (plus sixth-order
    isotropy for D3Q27, which has one more class) -- solved here with a
    linear solve and compared with the oracle's table."""
    e, w = orc.velocity_set(q)
    cls = np.abs(e).sum(1)
    classes = sorted(set(cls.tolist()))
    # conditions on the per-class weights: sum w, sum w ex^2, sum w ex^2 ey^2,
    # and (D3Q27) sum w ex^2 ey^2 ez^2 = cs^6
    rows, rhs = [], []
    ex2 = e[:, 0] ** 2
    ey2 = e[:, 1] ** 2
    ez2 = e[:, 2] ** 2
    for f, target in [(np.ones(q), 1.0), (ex2, CS2), (ex2 * ey2, CS2 ** 2)] + (
            [(ex2 * ey2 * ez2, CS2 ** 3)] if q == 27 else []):
        rows.append([f[cls == c].sum() for c in classes])
        rhs.append(target)
    A = np.array(rows, dtype=np.float64)
    sol = np.linalg.solve(A, np.array(rhs))
    for c, wc in zip(classes, sol):
        assert np.allclose(w[cls == c], wc, rtol=0, atol=1e-15)


@pytest.mark.parametrize("q", [15, 27])
def test_gamma_moments(q):
    """P2: sum Gamma = 1, sum Gamma e = u, sum Gamma e e = cs^2 I + u u."""
    e, w = orc.velocity_set(q)
    rng = np.random.default_rng(7)
    for _ in range(5):
        u = 0.05 * rng.standard_normal(3)
        G = orc.gamma(q, u)
        assert abs(G.sum() - 1.0) < 1e-15
        assert np.abs(G @ e - u).max() < 1e-16
        m2 = np.einsum("i,ia,ib->ab", G, e.astype(float), e.astype(float))
        assert np.abs(m2 - (CS2 * np.eye(3) + np.outer(u, u))).max() < 1e-15
    assert np.abs(orc.gamma(q, np.zeros(3)) - w).max() == 0.0


def test_hydro_equilibrium_moments():
    """P2: g_eq = p* w + (Gamma - w) has sum p* and first moment u."""
    e, w = orc.velocity_set(27)
    rng = np.random.default_rng(8)
    for _ in range(5):
        u = 0.05 * rng.standard_normal(3)
        ps = 1e-3 * rng.standard_normal()
        geq = orc.hydro_equilibrium(ps, u)
        assert abs(geq.sum() - ps) < 1e-16
        assert np.abs(geq @ e - u).max() < 1e-16


def test_phase_forcing_identities():
    """P3 (local): sum_i F^phi_i = 0 and sum_i F^phi_i e_i = cs^2 theta n,
    so the forcing conserves phi and carries the Allen-Cahn counter-flux."""
    e, w = orc.velocity_set(15)
    rng = np.random.default_rng(9)
    for _ in range(5):
        n = rng.standard_normal(3)
        n /= np.linalg.norm(n)
        theta = rng.uniform(0, 0.25)
        F = orc.phase_forcing(theta, n)
        assert abs(F.sum()) < 1e-17
        assert np.abs(F @ e - CS2 * theta * n).max() < 1e-16


def test_moment_matrix_weighted_orthogonal():
    """The D3Q27 moment basis: rows orthogonal under sum_i w_i, degrees
    0,1,2 occupy 1,3,6 rows, rows 1..3 are e_x, e_y, e_z, and M^-1 M = I."""
    e, w = orc.velocity_set(27)
    M, Mi, deg = orc.moment_matrix()
    G = (M * w) @ M.T
    off = G - np.diag(np.diag(G))
    assert np.abs(off).max() < 1e-14
    assert list(np.bincount(deg)) == [1, 3, 6, 7, 6, 3, 1]
    assert np.all(M[0] == 1.0)
    assert np.abs(M[1:4] - e.T).max() == 0.0
    assert np.abs(Mi @ M - np.eye(27)).max() < 1e-13


def _closed_form(g, u, F, rho, s):
    """g* = g_eq(u) + F_i/2 + (1 - s) w_i/(2 cs^4) (e e - cs^2 I):(Pi - p* cs^2 I - u u),
    the projection form of the weighted-orthogonal MRT with s on the six
    second-order moments and 1 elsewhere."""
    e, w = orc.velocity_set(27)
    e = e.astype(float)
    ps = g.sum()
    Pi = np.einsum("i,ia,ib->ab", g, e, e)
    A = Pi - ps * CS2 * np.eye(3) - np.outer(u, u)
    Hab = np.einsum("ia,ib->iab", e, e) - CS2 * np.eye(3)
    Fi = w * (e @ F) / (rho * CS2)
    geq = ps * w + orc.gamma(27, u) - w
    return geq + 0.5 * Fi + (1.0 - s) * w / (2 * CS2 * CS2) * np.einsum("iab,ab->i", Hab, A)


def test_mrt_collision_closed_form():
    """P4: the literal moment-space collision M^-1[m - S(m - m_eq + F_m/2) + F_m]
    equals the closed projection form; its zeroth moment is p* and its first
    moment j + F/rho."""
    e, w = orc.velocity_set(27)
    rng = np.random.default_rng(10)
    for s in (0.3, 2.0 / 3.0, 1.0, 1.25, 1.887):
        g = w * (1 + 0.2 * rng.standard_normal(27)) + 1e-3 * rng.standard_normal(27)
        ps = g.sum()
        j = g @ e
        F = 1e-3 * rng.standard_normal(3)
        rho = rng.uniform(0.001, 10)
        u = j + F / (2 * rho)
        out = orc.mrt_collide(g, ps, u, F, rho, s)
        assert np.abs(out - _closed_form(g, u, F, rho, s)).max() < 1e-14
        assert abs(out.sum() - ps) < 1e-14
        assert np.abs(out @ e - (j + F / rho)).max() < 1e-14


def test_viscous_bracket_identity():
    """P5: sum_k e_k e_k^T (Omega (g - g_eq(p*, u)))_k = s (Pi - p* cs^2 I - u u)."""
    e, w = orc.velocity_set(27)
    e = e.astype(float)
    rng = np.random.default_rng(11)
    for s in (0.5, 1.0, 1.6):
        g = w * (1 + 0.2 * rng.standard_normal(27))
        u = 0.05 * rng.standard_normal(3)
        ps = g.sum()
        Pi = np.einsum("i,ia,ib->ab", g, e, e)
        expect = s * (Pi - ps * CS2 * np.eye(3) - np.outer(u, u))
        assert np.abs(orc.viscous_bracket(g, s, u) - expect).max() < 1e-14


def _poly_field(n, coef):
    z, y, x = np.meshgrid(*[np.arange(n, dtype=float)] * 3, indexing="ij")
    c0, cx, cy, cz, cxx, cyy, czz, cxy, cxz, cyz = coef
    phi = (c0 + cx * x + cy * y + cz * z + cxx * x * x + cyy * y * y + czz * z * z
           + cxy * x * y + cxz * x * z + cyz * y * z)
    return phi


@pytest.mark.parametrize("q", [15, 27])
def test_stencils_exact_on_quadratics(q):
    """P6: the isotropic gradient and Laplacian are exact on quadratic
    polynomials at interior points (no wrap involved)."""
    n = 8
    P = orc.Params(nx=n, ny=n, nz=n)
    rng = np.random.default_rng(12)
    coef = rng.standard_normal(10) * 0.01
    phi = _poly_field(n, coef)
    c0, cx, cy, cz, cxx, cyy, czz, cxy, cxz, cyz = coef
    for (x, y, z) in [(3, 4, 2), (1, 1, 1), (6, 5, 4)]:
        grad, lap = orc.stencil(P, phi, q, x, y, z)
        ex = [cx + 2 * cxx * x + cxy * y + cxz * z,
              cy + 2 * cyy * y + cxy * x + cyz * z,
              cz + 2 * czz * z + cxz * x + cyz * y]
        assert np.abs(grad - ex).max() < 1e-13
        assert abs(lap - 2 * (cxx + cyy + czz)) < 1e-13


@pytest.mark.parametrize("q", [15, 27])
def test_stencils_second_order_convergence(q):
    """P6: on phi = sin(2 pi x / L) (periodic) the relative gradient and
    Laplacian errors fall with slope 2 in L."""
    errs_g, errs_l = [], []
    Ls = [16, 32, 64]
    for L in Ls:
        P = orc.Params(nx=L, ny=4, nz=4)
        x = np.arange(L, dtype=float)
        k = 2 * np.pi / L
        phi = np.broadcast_to(np.sin(k * (x + 0.3)), (4, 4, L)).copy()
        eg, el = 0.0, 0.0
        for xs in range(L):
            grad, lap = orc.stencil(P, phi, q, xs, 1, 2)
            eg = max(eg, abs(grad[0] - k * np.cos(k * (xs + 0.3))))
            el = max(el, abs(lap + k * k * np.sin(k * (xs + 0.3))))
            assert abs(grad[1]) < 1e-15 and abs(grad[2]) < 1e-15
        # relative to the amplitude of the exact derivative
        errs_g.append(eg / k)
        errs_l.append(el / (k * k))
        # in 1D both stencils reduce to the central differences, whose
        # leading errors are k^3/6 and k^4/12
        assert abs(eg / k ** 3 - 1.0 / 6.0) < 0.02
        assert abs(el / k ** 4 - 1.0 / 12.0) < 0.01
    for errs in (errs_g, errs_l):
        slope = np.polyfit(np.log(Ls), np.log(errs), 1)[0]
        assert -2.1 < slope < -1.9


def test_stencil_wall_mirror():
    """With y walls, a field that is even about the wall plane (y = 1/2)
    has zero normal gradient at the first fluid row: the wall row is read
    as the mirror image of the fluid row."""
    n = 8
    P = orc.Params(nx=n, ny=n, nz=n, walls_y=True)
    rng = np.random.default_rng(13)
    prof = rng.standard_normal(n)
    phi = np.broadcast_to(prof[None, :, None], (n, n, n)).copy()
    phi[:, 0, :] = 123.0   # wall row content must never be read
    phi[:, -1, :] = -77.0
    for y in (1, n - 2):
        grad, lap = orc.stencil(P, phi, 27, 3, y, 3)
        inner = y + 1 if y == 1 else y - 1
        d = prof[inner] - prof[y]
        sgn = 1.0 if y == 1 else -1.0
        # only the inner neighbour row differs from the centre: with the
        # mirror, the y-gradient is (1/2) * one-sided difference
        assert abs(grad[1] - sgn * 0.5 * d) < 1e-13
        assert abs(grad[0]) < 1e-15 and abs(grad[2]) < 1e-15
        assert abs(lap - d) < 1e-13
