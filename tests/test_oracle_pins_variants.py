"""Pins of the oracle's two model variants: the weakly compressible
equilibrium of Eq. (feq) and the modified nodal bounce-back of Sec. 2.2
(Eq. (bb) applied on wall nodes that also collide).

As in the main pin file, none of these re-type the oracle's formulas: they
check moments and conservation laws the variants must have, an exact
scaling symmetry that only the compressible form has, and closed-form
steady channel flows.
"""
import math

import numpy as np
import pytest

import oracle
from test_oracle_pins import _d2q9_shear_decay

LATTICES = [oracle.D2Q9, oracle.D3Q19, oracle.D3Q27]


def _dim(lattice):
    return 2 if lattice == oracle.D2Q9 else 3


@pytest.mark.parametrize("lattice", LATTICES)
def test_compressible_equilibrium_moments(lattice):
    """Eq. (feq): sum feq = rho, sum e feq = rho u and
    sum e e feq = rho c_s^2 I + rho u u with c_s^2 = 1/3."""
    e, t = oracle.lattice_tables(lattice)
    D = _dim(lattice)
    ef = e[:, :D].astype(float)
    rng = np.random.default_rng(15)
    for _ in range(20):
        rho = 1.0 + 0.3 * rng.uniform(-1, 1)
        u = np.zeros(3)
        u[:D] = 0.08 * rng.standard_normal(D)
        feq = oracle.equilibrium_node(lattice, rho, u, compressible=True)
        assert abs(feq.sum() - rho) < 1e-15
        assert np.abs(ef.T @ feq - rho * u[:D]).max() < 2e-16
        second = np.einsum("a,ai,aj->ij", feq, ef, ef)
        want = rho / 3 * np.eye(D) + rho * np.outer(u[:D], u[:D])
        assert np.abs(second - want).max() < 8e-16


@pytest.mark.parametrize("lattice", LATTICES)
@pytest.mark.parametrize("tau", [0.52, 0.8, 1.6])
def test_compressible_collision_conserves_mass_and_adds_F(lattice, tau):
    """With u = (j + F/2)/rho the collision still keeps sum f and adds
    exactly F to sum e f, now at densities far from 1."""
    e, t = oracle.lattice_tables(lattice)
    D = _dim(lattice)
    ef = e[:, :D].astype(float)
    rng = np.random.default_rng(int(tau * 100) + 7 * lattice)
    for _ in range(10):
        rho = 1.0 + 0.3 * rng.uniform(-1, 1)
        u = np.zeros(3)
        u[:D] = 0.05 * rng.standard_normal(D)
        f = oracle.equilibrium_node(lattice, rho, u, True) + 0.01 * t * rng.standard_normal(len(t))
        F = np.zeros(3)
        F[:D] = 1e-4 * rng.standard_normal(D)
        fb = oracle.collide_node(lattice, tau, F, f, compressible=True)
        assert abs(fb.sum() - f.sum()) <= 1e-15
        assert np.abs(ef.T @ fb - ef.T @ f - F[:D]).max() <= 2e-16
        # equilibrium at (rho, u) is a fixed point of the unforced collision
        feq = oracle.equilibrium_node(lattice, rho, u, True)
        assert np.abs(oracle.collide_node(lattice, tau, np.zeros(3), feq, True) - feq).max() < 1e-15


@pytest.mark.parametrize("lattice", LATTICES)
def test_compressible_update_is_homogeneous_of_degree_one(lattice):
    """Eq. (feq) is rho times a function of u, and u = (j + F/2)/rho, so
    scaling f and F by c scales the collided state by c.  The incompressible
    form, whose constant rho0 sets a scale, lacks this symmetry (control)."""
    e, t = oracle.lattice_tables(lattice)
    D = _dim(lattice)
    rng = np.random.default_rng(3 + lattice)
    c = 2.5
    for _ in range(10):
        u = np.zeros(3)
        u[:D] = 0.05 * rng.standard_normal(D)
        f = oracle.equilibrium_node(lattice, 1.1, u, True) + 0.01 * t * rng.standard_normal(len(t))
        F = np.zeros(3)
        F[:D] = 1e-4 * rng.standard_normal(D)
        a = oracle.collide_node(lattice, 0.7, F, f, compressible=True)
        b = oracle.collide_node(lattice, 0.7, c * F, c * f, compressible=True)
        assert np.abs(b - c * a).max() < 1e-15
        ai = oracle.collide_node(lattice, 0.7, F, f)
        bi = oracle.collide_node(lattice, 0.7, c * F, c * f)
        assert np.abs(bi - c * ai).max() > 1e-6


def test_compressible_run_is_homogeneous_and_matches_incompressible_at_unit_density():
    """Whole runs: (i) scaling the initial populations and F by c scales every
    later state by c (walls and propagation are linear); (ii) at a node with
    sum f = 1 the two equilibria coincide, so a run that starts from rest at
    rho = 1 with F = 0 stays identical in both models."""
    dims = (7, 6, 5)
    nx, ny, nz = dims
    rng = np.random.default_rng(21)
    rho = 1.0 + 0.02 * rng.standard_normal((nz, ny, nx))
    u = 0.03 * rng.standard_normal((3, nz, ny, nx))
    F = (2e-5, -1e-5, 1e-5)
    c = 1.75
    a = oracle.Sim(oracle.D3Q19, *dims, tau=0.7, force=F, bc=(0, 1, 2), compressible=True)
    a.init_equilibrium(rho, u)
    f0 = a.get_populations()
    a.step(15)
    b = oracle.Sim(oracle.D3Q19, *dims, tau=0.7, force=tuple(c * x for x in F), bc=(0, 1, 2),
                   compressible=True)
    b.set_populations(c * f0)
    b.step(15)
    assert np.abs(b.get_populations() - c * a.get_populations()).max() < 1e-15
    ra, ua = a.moments()
    rb, ub = b.moments()
    assert np.abs(ub - ua).max() < 1e-15 and np.abs(rb - c * ra).max() < 1e-14

    one = np.ones((nz, ny, nx))
    zero = np.zeros((3, nz, ny, nx))
    runs = []
    for comp in (False, True):
        s = oracle.Sim(oracle.D3Q19, *dims, tau=0.7, bc=(0, 1, 2), compressible=comp)
        s.init_equilibrium(one, zero)
        s.step(5)
        runs.append(s.get_populations())
    assert np.array_equal(runs[0], runs[1])


def _halfway_poiseuille(y, y1, y2, g, tau):
    """Steady forced channel between halfway bounce-back walls at y1, y2
    (BGK + trapezoidal forcing): (g/2nu)(y - y1)(y2 - y) + g(16L - 3)/(24nu),
    L = (tau - 1/2)^2."""
    nu = (tau - 0.5) / 3
    return g / (2 * nu) * (y - y1) * (y2 - y) + g * (16 * (tau - 0.5) ** 2 - 3) / (24 * nu)


@pytest.mark.parametrize("lattice", LATTICES)
@pytest.mark.parametrize("rho", [0.7, 1.5])
def test_compressible_poiseuille_velocity_is_force_over_density(lattice, rho):
    """At uniform density rho the compressible model's momentum rho u obeys
    the incompressible model's equations, so a channel driven by the force
    density F = rho g has the profile of the acceleration g; the
    incompressible model (rho0 = 1) gives rho times that (control)."""
    H, g, tau = 16, 1e-6, 0.9
    ny = H + 2
    y = np.arange(ny, dtype=float)
    want = _halfway_poiseuille(y, 0.5, H + 0.5, g, tau)
    nu = (tau - 0.5) / 3
    steps = int(math.log(1e13) / (nu * (math.pi / H) ** 2)) + 1
    got = {}
    for comp in (True, False):
        s = oracle.Sim(lattice, 1, ny, 1, tau=tau, force=(rho * g, 0, 0), bc=(0, 1, 0),
                       compressible=comp)
        s.init_equilibrium(np.full((1, ny, 1), rho), np.zeros((3, 1, ny, 1)))
        s.step(steps)
        r, u = s.moments()
        fl = s.geometry()[0, :, 0].astype(bool)
        got[comp] = u[0, 0, :, 0][fl]
        if comp:
            assert np.abs(r[0, :, 0][fl] - rho).max() < 1e-12
    w = want[1:-1]
    assert np.abs(got[True] - w).max() / w.max() < 1e-8
    assert np.abs(got[False] - rho * w).max() / w.max() < 1e-8


def test_compressible_taylor_green_decay_rate():
    """Shear waves decay at the rate of the linearised D2Q9 step (the same
    eigenvalue as in the incompressible model, whose linearisation about
    rest is identical) in the compressible model too: 2D Taylor-Green,
    D2Q9 128^2, tau = 0.8, small amplitude."""
    n, tau, U0 = 128, 0.8, 0.0025
    k = 2 * math.pi / n
    x = 2 * math.pi * np.arange(n) / n
    X, Y = x[None, None, :], x[None, :, None]
    u = np.zeros((3, 1, n, n))
    u[0] = U0 * np.sin(X) * np.cos(Y)
    u[1] = -U0 * np.cos(X) * np.sin(Y)
    rho = np.broadcast_to(1.0 + 3.0 * (U0 * U0 / 4.0) * (np.cos(2 * X) + np.cos(2 * Y)),
                          (1, n, n))
    s = oracle.Sim(oracle.D2Q9, n, n, 1, tau=tau, compressible=True)
    s.init_equilibrium(np.ascontiguousarray(rho), u)
    ts, ke = [], []
    for it in range(1001):
        if it % 10 == 0 and it >= 100:
            ts.append(it)
            ke.append(s.reduce()["ke"])
        if it < 1000:
            s.step(1)
    rate = -np.polyfit(np.array(ts, float), np.log(np.array(ke)), 1)[0]
    assert abs(rate / (2 * _d2q9_shear_decay(k, tau)) - 1) < 5e-6


def _nodal_poiseuille(y, H, g, tau):
    """Steady forced channel with walls on the nodes y = 0 and y = H of the
    modified nodal bounce-back (Eq. (bb) on wall nodes that collide), BGK
    with trapezoidal forcing, derived by hand from the steady state of the
    populations that are odd in e along the flow: in the bulk u'' = -g/nu
    exactly; on a wall node the rule f_a = f_abar for the unknown
    populations gives u + (tau - 1/2) g = 3 tau g there.  Hence
      u(y) = (g/2nu) y (H - y) + (2 tau + 1/2) g,
    a parabola through walls at the nodes plus a slip of O(g), i.e. second
    order relative to the O(g H^2/nu) flow."""
    nu = (tau - 0.5) / 3
    return g / (2 * nu) * y * (H - y) + (2 * tau + 0.5) * g


@pytest.mark.parametrize("lattice", LATTICES)
@pytest.mark.parametrize("tau", [0.6, 0.9, 1.5])
def test_nodal_bounce_back_poiseuille_closed_form(lattice, tau):
    H, g = 16, 1e-6
    ny = H + 1
    s = oracle.Sim(lattice, 1, ny, 1, tau=tau, force=(g, 0, 0), bc=(0, oracle.WALLS_NODAL, 0))
    assert s.geometry().all()  # wall nodes are fluid nodes that collide
    s.init_equilibrium(np.ones((1, ny, 1)), np.zeros((3, 1, ny, 1)))
    nu = (tau - 0.5) / 3
    steps = int(math.log(1e13) / (nu * (math.pi / H) ** 2)) + 1
    s.step(steps)
    _, u = s.moments()
    want = _nodal_poiseuille(np.arange(ny, dtype=float), H, g, tau)
    assert np.abs(u[0, 0, :, 0] - want).max() / want.max() < 1e-8
    assert np.abs(u[1]).max() < 1e-14


@pytest.mark.parametrize("axis,flow", [(0, 1), (2, 0), (2, 1)])
def test_nodal_bounce_back_on_every_axis(axis, flow):
    """The same closed form with the nodal walls across x or z and the force
    along another axis (D3Q19)."""
    H, g, tau = 12, 1e-6, 0.8
    n = [1, 1, 1]
    n[axis] = H + 1
    bc = [0, 0, 0]
    bc[axis] = oracle.WALLS_NODAL
    F = [0.0, 0.0, 0.0]
    F[flow] = g
    s = oracle.Sim(oracle.D3Q19, *n, tau=tau, force=F, bc=bc)
    shape = (n[2], n[1], n[0])
    s.init_equilibrium(np.ones(shape), np.zeros((3,) + shape))
    nu = (tau - 0.5) / 3
    s.step(int(math.log(1e13) / (nu * (math.pi / H) ** 2)) + 1)
    _, u = s.moments()
    prof = u[flow].reshape(-1)
    want = _nodal_poiseuille(np.arange(H + 1, dtype=float), H, g, tau)
    assert np.abs(prof - want).max() / want.max() < 1e-8


def test_nodal_unknowns_follow_eq_bb_and_rest_is_a_fixed_point():
    """After every propagation the unknown populations of a wall node equal
    the opposite ones (Eq. (bb)); values given for them on input are
    replaced; a uniform rest state at any density is a fixed point."""
    dims = (5, 6, 4)
    nx, ny, nz = dims
    e, t = oracle.lattice_tables(oracle.D3Q19)
    rng = np.random.default_rng(4)
    s = oracle.Sim(oracle.D3Q19, *dims, tau=0.7, force=(1e-5, 0, 2e-5), bc=(0, 3, 0))
    f = t[:, None, None, None] * (1 + 0.01 * rng.standard_normal((19, nz, ny, nx)))
    s.set_populations(f)
    for _ in range(3):
        g = s.get_populations()
        for a in range(19):
            ab = 18 - a
            if e[a][1] == 1:  # source beyond the wall y = 0
                assert np.array_equal(g[a, :, 0, :], g[ab, :, 0, :])
            if e[a][1] == -1:  # source beyond the wall y = ny - 1
                assert np.array_equal(g[a, :, -1, :], g[ab, :, -1, :])
        s.step(1)
    r = oracle.Sim(oracle.D3Q19, *dims, tau=0.7, bc=(0, 3, 0))
    r.init_equilibrium(np.full((nz, ny, nx), 1.3), np.zeros((3, nz, ny, nx)))
    f0 = r.get_populations()
    r.step(7)
    assert np.abs(r.get_populations() - f0).max() < 1e-14  # rounding of sum f only


def test_nodal_walls_validation():
    """At most one axis carries nodal walls (on a shared edge the unknowns
    would be defined by each other); a nodal axis needs three nodes."""
    with pytest.raises(ValueError):
        oracle.Sim(oracle.D3Q19, 4, 5, 6, tau=0.7, bc=(0, 3, 3))
    with pytest.raises(ValueError):
        oracle.Sim(oracle.D3Q19, 4, 2, 6, tau=0.7, bc=(0, 3, 0))
    oracle.Sim(oracle.D3Q19, 4, 5, 6, tau=0.7, bc=(1, 3, 2)).close()
