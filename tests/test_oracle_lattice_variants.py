"""Pins of the oracle's collision and stencil variants (the stencil study of
Sec. 5.1 and the D3Q19 validation lattice of Sec. 6.1): weighted-orthogonal
moment sets of D3Q15 and D3Q19, their moment-space collision against the
closed projection form, the raw-moment MRT of the phase field (Sec. 3.1),
and whole steps on the other lattice pairs against the physics the model
must reproduce.  None of the expected values comes from the oracle.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2012_06144_amd import inputs

CS2 = 1.0 / 3.0
EPS64 = np.finfo(np.float64).eps


@pytest.mark.parametrize("q,counts", [(15, [1, 3, 6, 4, 1]), (19, [1, 3, 6, 6, 3]),
                                      (27, [1, 3, 6, 7, 6, 3, 1])])
def test_moment_sets(q, counts):
    """The monomials x^a y^b z^c that are independent on the q-velocity set,
    by degree (for D3Q19: no xyz, and x^2 yz = yz... drop out), orthogonal
    under sum_i w_i f_i g_i; rows 1..3 are e_x, e_y, e_z themselves."""
    e, w = orc.velocity_set(q)
    M, Mi, R, Ri, deg, ex = orc.moment_matrix_q(q)
    assert np.bincount(deg).tolist() == counts
    G = (M * w[None, :]) @ M.T
    assert np.abs(G - np.diag(np.diag(G))).max() < 1e-14
    assert np.abs(M @ Mi - np.eye(q)).max() < 1e-13
    assert np.abs(R @ Ri - np.eye(q)).max() < 1e-13
    for k in range(1, 4):
        a = int(np.argmax(ex[k]))
        assert np.array_equal(M[k], e[:, a].astype(float))
    # raw rows are the monomials evaluated on the set
    for k in range(q):
        assert np.array_equal(R[k], np.prod(e.astype(float) ** ex[k][None, :], axis=1))


def _closed_form(e, w, g, pstar, u, F, rho, s):
    """g* = g_eq(u) + F_i/2 + (1 - s) w_i/(2 cs^4) (e_i e_i - cs^2 I) : A,
    A = Pi - p* cs^2 I - u u^T, F_i = w_i e_i.F/(rho cs^2) (Sec. 3.2 with all
    second-order moments at rate s and the rest at 1)."""
    e = e.astype(float)
    eu = e @ u
    geq = pstar * w + w * (eu / CS2 + eu ** 2 / (2 * CS2 ** 2) - u @ u / (2 * CS2))
    Pi = np.einsum("i,ia,ib->ab", g, e, e)
    A = Pi - pstar * CS2 * np.eye(3) - np.outer(u, u)
    H2 = np.einsum("ia,ib->iab", e, e) - CS2 * np.eye(3)[None]
    Fi = w * (e @ F) / (rho * CS2)
    return geq + 0.5 * Fi + (1 - s) * w / (2 * CS2 ** 2) * np.einsum("iab,ab->i", H2, A), A


@pytest.mark.parametrize("q", [15, 19])
def test_mrt_equals_closed_form(q):
    """P4 on the other hydrodynamic lattices: the literal M^-1 S M collision
    with the weighted-orthogonal set equals the closed projection form, and
    the viscous bracket is s (Pi - p* cs^2 I - u u^T) (P5)."""
    rng = np.random.default_rng(q)
    e, w = orc.velocity_set(q)
    for _ in range(5):
        u = 0.05 * rng.standard_normal(3)
        pstar = 1e-2 * rng.standard_normal()
        g = orc.hydro_equilibrium_q(q, pstar, u) + 1e-3 * rng.standard_normal(q) * w
        ps = g.sum()
        F = 1e-4 * rng.standard_normal(3)
        rho, s = 0.7, 1.3
        lit = orc.mrt_collide_q(q, g, ps, u, F, rho, s)
        cf, A = _closed_form(e, w, g, ps, u, F, rho, s)
        assert np.abs(lit - cf).max() < 1e-15
        V = orc.viscous_bracket_q(q, g, s, u)
        assert np.abs(V - s * A).max() < 1e-15


@pytest.mark.parametrize("q", [15, 19, 27])
def test_phase_mrt_relaxes_first_moments_only(q):
    """Raw-moment MRT of the phase field (Sec. 3.1): after the collision the
    zeroth moment is phi, the first-order moments are those of
    h + omega (h_eq - h - F/2) + F, every other raw moment is that of
    h_eq + F/2 (relaxed by one); with omega = 1 it is the SRT collision."""
    rng = np.random.default_rng(3 + q)
    e, w = orc.velocity_set(q)
    M, Mi, R, Ri, deg, ex = orc.moment_matrix_q(q)
    e = e.astype(float)
    phi, u = 0.6, 0.03 * rng.standard_normal(3)
    heq = phi * orc.gamma(q, u)
    h = heq + 0.01 * rng.standard_normal(q) * w
    h += (phi - h.sum()) / q                                # same zeroth moment
    n = rng.standard_normal(3)
    n /= np.linalg.norm(n)
    F = 0.2 * w * (e @ n)                                    # theta w_i e_i.n
    for omega in (1.7, 1.0):
        out = orc.phase_mrt_collide_q(q, h, heq, F, omega)
        assert abs(out.sum() - phi) < 1e-15
        j_expect = e.T @ (h + omega * (heq - h - 0.5 * F) + F)
        assert np.abs(e.T @ out - j_expect).max() < 1e-15
        other = [k for k in range(q) if deg[k] != 1]
        assert np.abs((R @ out)[other] - (R @ (heq + 0.5 * F))[other]).max() < 1e-15
        if omega == 1.0:
            assert np.abs(out - (heq + 0.5 * F)).max() < 1e-15


PAIRS = [(19, 19, False), (27, 27, False), (15, 27, True)]


def _p(s, qp, qh, mrt):
    return orc.Params(**s.physics(), lattice_phase=qp, lattice_hydro=qh, phase_mrt=mrt)


@pytest.mark.parametrize("qp,qh,mrt", PAIRS)
def test_mass_conserved_other_lattices(qp, qh, mrt):
    """sum(phi) exact to rounding, periodic and between walls while a bubble rises."""
    for s in (inputs.static_droplet(n=16, R=5.0, noise=1e-5),
              inputs.rising_bubble(12, 30, 12, D=8.0, center=(6.0, 10.0, 6.0), g=2e-5)):
        phi, u, ps = inputs.build_fields(s)
        o = orc.Oracle(_p(s, qp, qh, mrt))
        o.init(phi, u, ps)
        m0 = o.stats()["mass"]
        o.step(200)
        assert abs(o.stats()["mass"] - m0) / m0 <= 4 * EPS64 * 200


@pytest.mark.parametrize("qp,qh,mrt", PAIRS)
def test_flat_interface_other_lattices(qp, qh, mrt):
    """The planar profile stays the tanh of Sec. 3.1 (within the discrete
    profile's 6e-3 at xi = 4) with width xi, and stays planar."""
    nx, xi = 64, 4.0
    x = np.arange(nx, dtype=float)
    a, b = nx / 4 - 0.5, 3 * nx / 4 - 0.5
    prof = np.minimum(0.5 + 0.5 * np.tanh(2 * (x - a) / xi), 0.5 + 0.5 * np.tanh(2 * (b - x) / xi))
    P = orc.Params(nx=nx, ny=2, nz=2, xi=xi, mobility=0.02, sigma=1e-3, rho_L=1.0, rho_H=10.0,
                   tau_L=1.0, tau_H=1.0, lattice_phase=qp, lattice_hydro=qh, phase_mrt=mrt)
    o = orc.Oracle(P)
    o.init(np.broadcast_to(prof, (2, 2, nx)).copy(), np.zeros((3, 2, 2, nx)), np.zeros((2, 2, nx)))
    o.step(3000)
    _, _, ph, _ = o.state()
    assert np.abs(ph[0, 0] - prof).max() < 6e-3
    assert abs(o.stats()["xi_eff"] / xi - 1.0) < 1e-2
    assert np.abs(ph - ph[0:1, 0:1, :]).max() < 1e-14


@pytest.mark.parametrize("qh", [19, 15])
def test_poiseuille_exact_other_lattices(qh):
    """Halfway bounce-back is exact for the body-force parabola at tau = 3/8
    on the other hydrodynamic lattices too."""
    ny, tau, a = 18, 0.375, 1e-6
    P = orc.Params(nx=1, ny=ny, nz=1, walls_y=True, rho_L=1.0, rho_H=1.0, tau_L=tau, tau_H=tau,
                   accel=(a, 0.0, 0.0), sigma=1e-4, xi=4.0, lattice_phase=qh, lattice_hydro=qh)
    phi = np.ones((1, ny, 1))
    phi[:, 0, :] = phi[:, -1, :] = 0.0
    o = orc.Oracle(P)
    o.init(phi, np.zeros((3, 1, ny, 1)), np.zeros((1, ny, 1)))
    o.step(20000)
    _, _, _, u = o.state()
    y = np.arange(ny, dtype=float)
    ex = a / (2 * tau / 3.0) * (y - 0.5) * (ny - 1.5 - y)
    f = slice(1, ny - 1)
    assert np.abs(u[0, 0, f, 0] - ex[f]).max() / ex[f].max() < 1e-9


@pytest.mark.parametrize("qp,qh,mrt", PAIRS)
def test_laplace_cylinder_other_lattices(qp, qh, mrt):
    """Pressure jump sigma / R of a heavy column (nz = 1), within 3 % at R = 8."""
    R, xi = 8.0, 4.0
    n = int(4 * R)
    P = orc.Params(nx=n, ny=n, nz=1, xi=xi, mobility=0.02, sigma=1e-3, rho_L=1.0, rho_H=10.0,
                   tau_L=1.0, tau_H=1.0, lattice_phase=qp, lattice_hydro=qh, phase_mrt=mrt)
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


@pytest.mark.parametrize("qp,qh,mrt", PAIRS)
def test_galilean_advection_other_lattices(qp, qh, mrt):
    """A density-matched bubble in a uniform stream moves by U t (1 %)."""
    U, steps = 0.02, 200
    s = inputs.Setup(name="adv", nx=32, ny=16, nz=16, walls_y=False, xi=4.0, mobility=0.02,
                     sigma=1e-4, rho_L=1.0, rho_H=1.0, tau_L=0.3, tau_H=0.3, kind="bubble",
                     radius=4.0, center=(8.0, 8.0, 8.0))
    phi, u, ps = inputs.build_fields(s)
    u[0][:] = U
    o = orc.Oracle(_p(s, qp, qh, mrt))
    o.init(phi, u, ps)
    c0 = np.array(o.stats()["centroid"])
    o.step(steps)
    c1 = np.array(o.stats()["centroid"])
    assert abs((c1[0] - c0[0]) / (U * steps) - 1.0) < 1e-2
    assert np.abs(c1[1:] - c0[1:]).max() < 1e-2
