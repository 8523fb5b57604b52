"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these re-type the oracle's formulas: each checks a property that the
paper's method must have (tables printed in Sec. 2.1, conservation by the
collision of Eq. (collision), streaming as the permutation of Eq.
(propagation), bounce-back of Eq. (bb), closed-form flows) so that a dropped
term, a sign or index slip, or a transposed operand in the oracle fails at
least one of them.
"""
import math
from fractions import Fraction
import os

import numpy as np
import pytest

import oracle
from paper_2201_11330_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def _load_golden_d2q9():
    rows = []
    with open(os.path.join(HERE, "golden", "d2q9_lattice.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            a, ex, ey, t = line.split()
            rows.append((int(a), int(ex), int(ey), float(Fraction(t))))
    return rows


def test_d2q9_tables_match_the_paper():
    e, t = oracle.lattice_tables(oracle.D2Q9)
    for a, ex, ey, tt in _load_golden_d2q9():
        assert (e[a, 0], e[a, 1], e[a, 2]) == (ex, ey, 0)
        assert t[a] == tt


@pytest.mark.parametrize("lattice", [oracle.D2Q9, oracle.D3Q19, oracle.D3Q27])
def test_lattice_symmetry_and_isotropy(lattice):
    """Opposite index m-1-a (Sec. 2.1) and the moment conditions that make the
    weights of Qian's DdQm models: sum t = 1, sum t e = 0, sum t e e = I/3,
    odd moments zero, sum t e_i e_j e_k e_l = (d_ij d_kl + d_ik d_jl + d_il d_jk)/9."""
    e, t = oracle.lattice_tables(lattice)
    Q = len(t)
    D = 2 if lattice == oracle.D2Q9 else 3
    for a in range(Q):
        assert np.all(e[Q - 1 - a] == -e[a])
    ef = e[:, :D].astype(float)
    I = np.eye(D)
    assert abs(t.sum() - 1.0) < 1e-15
    assert np.abs(np.einsum("a,ai->i", t, ef)).max() < 1e-15
    assert np.abs(np.einsum("a,ai,aj->ij", t, ef, ef) - I / 3).max() < 1e-15
    assert np.abs(np.einsum("a,ai,aj,ak->ijk", t, ef, ef, ef)).max() < 1e-15
    four = np.einsum("a,ai,aj,ak,al->ijkl", t, ef, ef, ef, ef)
    iso = (np.einsum("ij,kl->ijkl", I, I) + np.einsum("ik,jl->ijkl", I, I)
           + np.einsum("il,jk->ijkl", I, I)) / 9
    assert np.abs(four - iso).max() < 1e-15


def test_d3q27_velocity_set_and_weights():
    """D3Q27 = all of {-1,0,1}^3 in lexicographic order (e_x slowest), with
    the tensor-product weights (2/3, 1/6, 1/6)^3: 8/27, 2/27, 1/54, 1/216."""
    e, t = oracle.lattice_tables(oracle.D3Q27)
    want = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)]
    assert [tuple(v) for v in e] == want
    w1 = {0: 2 / 3, 1: 1 / 6, -1: 1 / 6}
    for a, v in enumerate(e):
        assert abs(t[a] - w1[v[0]] * w1[v[1]] * w1[v[2]]) < 1e-17


def test_d3q19_velocity_set_is_the_qian_set():
    """D3Q19 = rest + 6 faces + 12 edges of {-1,0,1}^3 (no corners), each once,
    in the lexicographic order (e_x slowest) that extends the D2Q9 numbering."""
    e, t = oracle.lattice_tables(oracle.D3Q19)
    want = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)
            if abs(a) + abs(b) + abs(c) <= 2]
    assert [tuple(v) for v in e] == want
    for a, v in enumerate(e):
        n = int(np.abs(v).sum())
        assert t[a] == {0: 1 / 3, 1: 1 / 18, 2: 1 / 36}[n]


@pytest.mark.parametrize("lattice", [oracle.D2Q9, oracle.D3Q19, oracle.D3Q27])
def test_incompressible_equilibrium_moments(lattice):
    """The incompressible equilibrium of Eq. (incompressible_feq) has
    sum feq = p/c_s^2, sum e feq = rho0 u and sum e e feq = (p/c_s^2) c_s^2 I
    + rho0 u u (He-Luo): these fix the constants 3, 4.5, 1.5 and the weights."""
    e, t = oracle.lattice_tables(lattice)
    D = 2 if lattice == oracle.D2Q9 else 3
    rng = np.random.default_rng(5)
    for _ in range(20):
        rho = 1.0 + 0.1 * rng.standard_normal()
        u = np.zeros(3)
        u[:D] = 0.05 * rng.standard_normal(D)
        feq = oracle.equilibrium_node(lattice, rho, u)
        ef = e[:, :D].astype(float)
        assert abs(feq.sum() - rho) < 1e-15
        assert np.abs(ef.T @ feq - u[:D]).max() < 1e-16
        second = np.einsum("a,ai,aj->ij", feq, ef, ef)
        want = rho / 3 * np.eye(D) + np.outer(u[:D], u[:D])
        assert np.abs(second - want).max() < 1e-15


def _random_pops(lattice, rng, amp=0.01):
    e, t = oracle.lattice_tables(lattice)
    D = 2 if lattice == oracle.D2Q9 else 3
    u = np.zeros(3)
    u[:D] = 0.05 * rng.standard_normal(D)
    return oracle.equilibrium_node(lattice, 1.0, u) + amp * t * rng.standard_normal(len(t))


@pytest.mark.parametrize("lattice", [oracle.D2Q9, oracle.D3Q19, oracle.D3Q27])
@pytest.mark.parametrize("tau", [0.51, 0.6, 0.8, 1.0, 1.7])
def test_collision_conserves_mass_and_adds_F_momentum(lattice, tau):
    """Pin P1: the collision keeps sum f exactly and changes sum e f by exactly
    F: -omega (j - rho0 u) + (1 - omega/2) F = omega F/2 + F - omega F/2."""
    e, t = oracle.lattice_tables(lattice)
    D = 2 if lattice == oracle.D2Q9 else 3
    rng = np.random.default_rng(int(tau * 100) + lattice)
    for _ in range(10):
        f = _random_pops(lattice, rng)
        F = np.zeros(3)
        F[:D] = 1e-5 * rng.standard_normal(D)
        fb = oracle.collide_node(lattice, tau, F, f)
        ef = e[:, :D].astype(float)
        # populations sum to about 1: a few units of roundoff of that sum
        assert abs(fb.sum() - f.sum()) <= 1e-15
        assert np.abs((ef.T @ fb) - (ef.T @ f) - F[:D]).max() <= 2e-16
        fb0 = oracle.collide_node(lattice, tau, np.zeros(3), f)
        assert np.abs((ef.T @ fb0) - (ef.T @ f)).max() <= 2e-16


@pytest.mark.parametrize("lattice", [oracle.D2Q9, oracle.D3Q19, oracle.D3Q27])
def test_collision_relaxes_toward_equilibrium(lattice):
    """Eq. (collision): the non-equilibrium part is scaled by (1 - omega) and
    equilibrium is a fixed point (pin P2)."""
    rng = np.random.default_rng(9)
    e, t = oracle.lattice_tables(lattice)
    D = 2 if lattice == oracle.D2Q9 else 3
    for tau in (0.55, 0.8, 1.3):
        u = np.zeros(3)
        u[:D] = 0.04 * rng.standard_normal(D)
        rho = 1.0 + 0.01 * rng.standard_normal()
        feq = oracle.equilibrium_node(lattice, rho, u)
        assert np.abs(oracle.collide_node(lattice, tau, np.zeros(3), feq) - feq).max() < 2e-16
        # A non-equilibrium part with zero mass and momentum relaxes by 1 - 1/tau.
        neq = rng.standard_normal(len(t)) * t * 1e-3
        ef = e[:, :D].astype(float)
        basis = np.vstack([np.ones(len(t)), ef.T])
        neq -= basis.T @ np.linalg.lstsq(basis.T, neq, rcond=None)[0]
        fb = oracle.collide_node(lattice, tau, np.zeros(3), feq + neq)
        assert np.abs(fb - (feq + (1 - 1 / tau) * neq)).max() < 2e-16


@pytest.mark.parametrize("lattice", [oracle.D2Q9, oracle.D3Q19, oracle.D3Q27])
def test_complex_collision_matches_real(lattice):
    """The complex instantiation used for derivatives equals the real one
    when imaginary parts are zero, and a complex step gives the directional
    derivative (checked against a central difference)."""
    rng = np.random.default_rng(3)
    f = _random_pops(lattice, rng)
    F = np.array([1e-5, -2e-5, 3e-5 if lattice == oracle.D3Q19 else 0.0])
    real = oracle.collide_node(lattice, 0.7, F, f)
    cplx = oracle.collide_node_complex(lattice, 0.7, F, f)
    assert np.array_equal(cplx.real, real) and np.all(cplx.imag == 0)
    d = rng.standard_normal(len(f))
    h = 1e-30
    cs = oracle.collide_node_complex(lattice, 0.7, F, f + 1j * h * d).imag / h
    eps = 1e-6
    fd = (oracle.collide_node(lattice, 0.7, F, f + eps * d)
          - oracle.collide_node(lattice, 0.7, F, f - eps * d)) / (2 * eps)
    assert np.abs(cs - fd).max() < 1e-8


def _equilibrium_state(lattice, dims, rho, u):
    s = oracle.Sim(lattice, *dims, tau=0.8)
    s.init_equilibrium(rho, u)
    return s.get_populations()


@pytest.mark.parametrize("lattice,dims", [(oracle.D2Q9, (9, 7, 1)), (oracle.D3Q19, (6, 5, 4)),
                                          (oracle.D3Q27, (5, 4, 6))])
def test_pure_streaming_is_a_shift(lattice, dims):
    """Pin P4: with omega = 0 (tau = +inf) and F = 0 one step is exactly
    Eq. (propagation): f_a(x, t) = f_a(x - e_a, t - 1) with periodic wrap."""
    rng = np.random.default_rng(1)
    nx, ny, nz = dims
    Q = {oracle.D2Q9: 9, oracle.D3Q19: 19, oracle.D3Q27: 27}[lattice]
    e, _ = oracle.lattice_tables(lattice)
    f0 = rng.uniform(0.0, 0.1, size=(Q, nz, ny, nx))
    s = oracle.Sim(lattice, nx, ny, nz, tau=math.inf)
    s.set_populations(f0)
    s.step(1)
    f1 = s.get_populations()
    for a in range(Q):
        want = np.roll(f0[a], shift=(e[a, 2], e[a, 1], e[a, 0]), axis=(0, 1, 2))
        assert np.array_equal(f1[a], want)


def test_pure_streaming_returns_after_n_steps():
    """Pin P4: n steps of pure streaming on a periodic n^3 cube are the
    identity, bit for bit."""
    rng = np.random.default_rng(2)
    n = 6
    f0 = rng.uniform(0.0, 0.1, size=(19, n, n, n))
    s = oracle.Sim(oracle.D3Q19, n, n, n, tau=math.inf)
    s.set_populations(f0)
    s.step(n - 1)
    assert not np.array_equal(s.get_populations(), f0)
    s.step(1)
    assert np.array_equal(s.get_populations(), f0)


@pytest.mark.parametrize("bc", [(0, 1, 0), (0, 2, 0), (1, 1, 1), (2, 0, 2)])
def test_pure_streaming_with_walls_is_a_reflecting_permutation(bc):
    """Eq. (bb) at halfway walls: with omega = 0 a population that runs into
    a wall comes back reversed one step later, so populations are only
    permuted (sum and multiset kept) and 2L steps along a 1D channel of L
    fluid nodes return the initial state."""
    rng = np.random.default_rng(4)
    dims = (5, 6, 4)
    nx, ny, nz = dims
    s = oracle.Sim(oracle.D3Q19, nx, ny, nz, tau=math.inf, bc=bc)
    fluid = s.geometry()
    f0 = rng.uniform(0.0, 0.1, size=(19, nz, ny, nx)) * fluid
    s.set_populations(f0)
    s.step(1)
    f1 = s.get_populations()
    assert np.array_equal(np.sort(f1[:, fluid].ravel()), np.sort(f0[:, fluid].ravel()))
    # A single population moving in +y towards the wall.
    L = 4
    s = oracle.Sim(oracle.D3Q19, 1, L + 2, 1, tau=math.inf, bc=(0, 1, 0))
    f = np.zeros((19, 1, L + 2, 1))
    f[12, 0, 2, 0] = 1.0  # e = (0, 1, 0)
    s.set_populations(f)
    s.step(L - 1)  # two steps up to the last fluid row y = L, one more to reflect there
    g = s.get_populations()
    assert g[6, 0, L, 0] == 1.0 and g.sum() == 1.0  # reversed (0,-1,0) at the last fluid row
    s.step(L + 1)
    assert np.array_equal(s.get_populations(), f)


@pytest.mark.parametrize("lattice,dims", [(oracle.D2Q9, (8, 6, 1)), (oracle.D3Q19, (5, 6, 4)),
                                          (oracle.D3Q27, (4, 5, 3))])
def test_uniform_equilibrium_is_a_fixed_point(lattice, dims):
    """Pin P3: a uniform equilibrium is left unchanged by a periodic step."""
    nx, ny, nz = dims
    u = np.zeros((3, nz, ny, nx))
    u[0], u[1] = 0.03, -0.02
    if lattice != oracle.D2Q9:
        u[2] = 0.01
    rho = np.full((nz, ny, nx), 1.02)
    s = oracle.Sim(lattice, nx, ny, nz, tau=0.7)
    s.init_equilibrium(rho, u)
    f0 = s.get_populations()
    s.step(5)
    assert np.abs(s.get_populations() - f0).max() < 1e-16


def _tg3(dims, seed=2):
    nx, ny, nz = dims
    rho, u = W.taylor_green_3d(nx, ny, nz, U0=0.05)
    noise = W.population_noise(W.D3Q19, dims, 1e-6, seed)
    return rho, u, noise


def test_translation_equivariance_bit_exact():
    """Pin P5: a periodically shifted input gives the shifted output."""
    dims = (7, 6, 5)
    nx, ny, nz = dims
    rho, u, noise = _tg3(dims)
    a = oracle.Sim(oracle.D3Q19, *dims, tau=0.6, force=(1e-6, 0, 2e-6))
    a.init_equilibrium(rho, u, noise)
    f0 = a.get_populations()
    a.step(4)
    shift = (2, 3, 1)
    b = oracle.Sim(oracle.D3Q19, *dims, tau=0.6, force=(1e-6, 0, 2e-6))
    b.set_populations(np.roll(f0, shift, axis=(1, 2, 3)))
    b.step(4)
    assert np.array_equal(b.get_populations(), np.roll(a.get_populations(), shift, axis=(1, 2, 3)))


def test_affine_equivariance_of_the_deviation_form():
    """Pin P6: the incompressible step commutes with f -> f - c t (the
    equilibrium is affine in sum f and sum t e = 0), which is what lets the
    populations be stored as deviations f - t."""
    dims = (6, 5, 4)
    rho, u, noise = _tg3(dims)
    _, t = oracle.lattice_tables(oracle.D3Q19)
    a = oracle.Sim(oracle.D3Q19, *dims, tau=0.6, force=(1e-6, -1e-6, 0), bc=(0, 1, 0))
    a.init_equilibrium(rho, u, noise)
    f0 = a.get_populations()
    fluid = a.geometry()
    b = oracle.Sim(oracle.D3Q19, *dims, tau=0.6, force=(1e-6, -1e-6, 0), bc=(0, 1, 0))
    b.set_populations(f0 - t[:, None, None, None] * fluid)
    a.step(10)
    b.step(10)
    diff = b.get_populations() + t[:, None, None, None] * fluid - a.get_populations()
    assert np.abs(diff).max() < 1e-15


@pytest.mark.parametrize("bc", [(0, 0, 0), (0, 1, 0), (2, 1, 1)])
def test_mass_conservation_and_momentum_growth(bc):
    """Pin P11: total mass is constant (collision keeps it and bounce-back only
    reverses populations); in a fully periodic box the total momentum grows
    by exactly V F per step."""
    dims = (6, 7, 5)
    nx, ny, nz = dims
    rho, u, noise = _tg3(dims)
    F = (2e-6, -1e-6, 5e-7)
    s = oracle.Sim(oracle.D3Q19, *dims, tau=0.65, force=F, bc=bc)
    fluid = s.geometry()
    s.init_equilibrium(rho, u, noise)
    e, _ = oracle.lattice_tables(oracle.D3Q19)
    f0 = s.get_populations()
    m0 = f0.sum()
    j0 = np.einsum("ad,azyx->d", e.astype(float), f0)
    n = 12
    s.step(n)
    f = s.get_populations()
    assert abs(f.sum() - m0) / m0 < 1e-14
    if bc == (0, 0, 0):
        j = np.einsum("ad,azyx->d", e.astype(float), f)
        V = fluid.sum()
        assert np.abs(j - j0 - n * V * np.asarray(F)).max() < 1e-15 * V
    red = s.reduce()
    assert abs(red["mass"] - f.sum()) < 1e-12 and red["nonfinite"] == 0


def test_moments_follow_postprocessing():
    """PostProcessing: rho = sum f and u = (sum e f + F/2)/rho0 at every node."""
    dims = (5, 4, 3)
    rho, u, noise = _tg3(dims)
    F = np.array([1e-5, 2e-5, -3e-5])
    s = oracle.Sim(oracle.D3Q19, *dims, tau=0.9, force=F)
    s.init_equilibrium(rho, u, noise)
    s.step(3)
    f = s.get_populations()
    r, v = s.moments()
    e, _ = oracle.lattice_tables(oracle.D3Q19)
    assert np.abs(r - f.sum(0)).max() < 1e-15
    j = np.einsum("ad,azyx->dzyx", e.astype(float), f)
    assert np.abs(v - (j + F[:, None, None, None] / 2)).max() < 1e-17


# Monitor (Sec. 3.6 Monitor listing): total mass, kinetic energy and the
# largest speed over the fluid nodes.  The pins below use states whose
# moments are known in closed form, so the sums have exact values; the
# listing's own loop starts at its second node and takes |u| in two
# dimensions, and neither quirk is a property of the method, so a skipped
# node, a 2-D norm or a dropped 1/2 must fail here.


@pytest.mark.parametrize("lattice,dims,bc", [
    (oracle.D2Q9, (7, 5, 1), (0, 0, 0)),
    (oracle.D3Q19, (5, 6, 4), (0, 0, 0)),
    (oracle.D3Q19, (5, 7, 4), (0, 1, 0)),
    (oracle.D3Q27, (4, 5, 6), (1, 0, 2)),
])
def test_monitor_of_a_uniform_flow(lattice, dims, bc):
    """A uniform equilibrium of density rho and velocity u = (a, b, c) (every
    component nonzero in 3D) has the moments rho and u at every fluid node
    (Sec. 2.1: the equilibrium's zeroth and first moments), so the Monitor
    must give mass = V rho, KE = (rho0/2) V |u|^2 with the 3-D norm and
    max |u| = |u|, V the number of fluid nodes.  After periodic steps the
    state is unchanged (Pin P3) and so are the three values."""
    nx, ny, nz = dims
    vel = np.array([0.031, -0.017, 0.0 if lattice == oracle.D2Q9 else 0.023])
    rho0 = 1.07
    s = oracle.Sim(lattice, nx, ny, nz, tau=0.7, bc=bc)
    fluid = s.geometry()
    V = int(fluid.sum())
    assert V < nx * ny * nz or bc == (0, 0, 0)
    u = np.zeros((3, nz, ny, nx))
    u[:, fluid] = vel[:, None]
    s.init_equilibrium(np.full((nz, ny, nx), rho0), u)
    speed = math.sqrt(float(vel @ vel))
    steps = [0, 3] if bc == (0, 0, 0) else [0]
    for n in steps:
        s.step(n)
        red = s.reduce()
        assert abs(red["mass"] - V * rho0) <= 1e-14 * V * rho0
        assert abs(red["ke"] - 0.5 * V * speed * speed) <= 1e-13 * V * speed * speed
        assert abs(red["umax"] - speed) <= 1e-14 * speed
        assert red["nonfinite"] == 0


def test_monitor_of_the_compressible_uniform_flow():
    """With the compressible equilibrium (Eq. (feq)) the kinetic energy is
    sum (rho/2)|u|^2: a uniform flow at rho = 1.5 gives 1.5 times the
    incompressible model's (rho0/2) V |u|^2, which the incompressible form of
    the sum would miss."""
    dims = (5, 4, 6)
    nx, ny, nz = dims
    vel = np.array([0.02, 0.015, -0.03])
    speed2 = float(vel @ vel)
    out = {}
    for comp, r in ((True, 1.5), (False, 1.5), (True, 0.6)):
        s = oracle.Sim(oracle.D3Q19, nx, ny, nz, tau=0.8, compressible=comp)
        u = np.broadcast_to(vel[:, None, None, None], (3, nz, ny, nx))
        s.init_equilibrium(np.full((nz, ny, nx), r), u)
        s.step(2)
        out[(comp, r)] = red = s.reduce()
        V = nx * ny * nz
        want = 0.5 * (r if comp else 1.0) * V * speed2
        assert abs(red["ke"] - want) <= 1e-13 * want
        assert abs(red["mass"] - r * V) <= 1e-14 * r * V
        assert abs(red["umax"] - math.sqrt(speed2)) <= 1e-14 * math.sqrt(speed2)
    assert abs(out[(True, 1.5)]["ke"] / out[(False, 1.5)]["ke"] - 1.5) < 1e-12


@pytest.mark.parametrize("dims", [(16, 16, 16), (16, 12, 8), (12, 20, 4)])
def test_monitor_of_the_taylor_green_start(dims):
    """The 3D Taylor-Green start u = U0 sin x cos y cos z, v = -U0 cos x
    sin y cos z, w = 0 on grids of n_i >= 3 nodes per axis: since
    sum_i sin^2(2 pi i/n) = sum_i cos^2(2 pi i/n) = n/2 and
    sum_i cos(4 pi i/n) = 0, the grid sums are exactly
    KE = (1/2) sum (u^2 + v^2) = U0^2 nx ny nz / 8 and mass = nx ny nz, and
    with every n_i divisible by 4 the largest speed is U0 (attained at
    x = pi/2, y = z = 0; sin^2 x cos^2 y + cos^2 x sin^2 y <= 1)."""
    nx, ny, nz = dims
    U0 = 0.05
    rho, u = W.taylor_green_3d(nx, ny, nz, U0=U0)
    s = oracle.Sim(oracle.D3Q19, nx, ny, nz, tau=0.6)
    s.init_equilibrium(rho, u)
    red = s.reduce()
    V = nx * ny * nz
    assert abs(red["ke"] - U0 * U0 * V / 8) <= 1e-13 * U0 * U0 * V
    assert abs(red["mass"] - V) <= 1e-14 * V
    assert abs(red["umax"] - U0) <= 1e-14 * U0


def test_monitor_counts_non_finite_populations():
    """The Monitor's non-finite count is the number of NaN or infinite
    populations on fluid nodes."""
    dims = (4, 5, 3)
    nx, ny, nz = dims
    s = oracle.Sim(oracle.D3Q19, nx, ny, nz, tau=0.7, bc=(0, 1, 0))
    rho, u = np.ones((nz, ny, nx)), np.zeros((3, nz, ny, nx))
    s.init_equilibrium(rho, u)
    f = s.get_populations()
    f[3, 1, 2, 1] = np.nan
    f[7, 2, 3, 0] = np.inf
    f[11, 0, 0, 2] = np.nan  # a solid node (row y = 0): not counted
    s.set_populations(f)
    assert s.reduce()["nonfinite"] == 2


def _ke_rate(lattice, dims, tau, steps, rho, u, every=10, skip=100):
    s = oracle.Sim(lattice, *dims, tau=tau)
    s.init_equilibrium(rho, u)
    ts, ke = [], []
    for it in range(steps + 1):
        if it % every == 0 and it >= skip:
            ts.append(it)
            ke.append(s.reduce()["ke"])
        if it < steps:
            s.step(1)
    slope = np.polyfit(np.array(ts, float), np.log(np.array(ke)), 1)[0]
    return -slope


def _d2q9_shear_decay(k, tau):
    """Decay per step of a small shear wave along the diagonal k(1,1): the
    modulus of the slowest non-conserved eigenvalue branch of the linearised
    D2Q9 step, brute force from the 9x9 operator built from the oracle's own
    collision Jacobian and the exact streaming phase."""
    e, t = oracle.lattice_tables(oracle.D2Q9)
    f0 = oracle.equilibrium_node(oracle.D2Q9, 1.0, np.zeros(3))
    h = 1e-30
    Jc = np.zeros((9, 9))
    for b in range(9):
        d = np.zeros(9)
        d[b] = 1.0
        Jc[:, b] = oracle.collide_node_complex(oracle.D2Q9, tau, 0.0, f0 + 1j * h * d).imag / h
    kv = np.array([k, k])
    S = np.diag(np.exp(-1j * (e[:, :2] @ kv)))
    lam = np.linalg.eigvals(S @ Jc)
    # The shear mode is the slowly decaying eigenvalue closest to 1 whose
    # eigenvector carries transverse momentum.
    w, V = np.linalg.eig(S @ Jc)
    khat = kv / np.linalg.norm(kv)
    perp = np.array([-khat[1], khat[0]])
    best = None
    for i in range(9):
        mom = e[:, :2].T @ V[:, i]
        if abs(perp @ mom) > 0.5 * np.linalg.norm(mom) and abs(w[i]) > 0.9:
            if best is None or abs(w[i]) > abs(best):
                best = w[i]
    assert best is not None, lam
    return -math.log(abs(best))


@pytest.mark.slow
def test_taylor_green_2d_decay_rate():
    """Pin P8 (workload D2Q9 128^2, tau = 0.8, 1000 steps): the kinetic energy
    of the 2D Taylor-Green vortex decays as exp(-2 nu k^2 t * 2) with
    nu = (tau - 1/2)/3 and k = 2 pi/128.  At small amplitude the measured rate
    converges to the brute-force eigenvalue of the linearised D2Q9 step (the
    gap at U0 = 0.01 is the O(Ma^2) nonlinear correction and shrinks 4x per
    halving of U0)."""
    n, tau = 128, 0.8
    nu = (tau - 0.5) / 3
    k = 2 * math.pi / n
    continuum = 4 * nu * k * k
    rho, u = W.taylor_green_2d(n, U0=0.01)
    rate = _ke_rate(oracle.D2Q9, (n, n, 1), tau, 1000, rho, u)
    assert abs(rate / continuum - 1) < 1e-4
    lattice_rate = 2 * _d2q9_shear_decay(k, tau)
    assert abs(rate / lattice_rate - 1) < 1e-4
    rho, u = W.taylor_green_2d(n, U0=0.0025)
    rate_small = _ke_rate(oracle.D2Q9, (n, n, 1), tau, 1000, rho, u)
    assert abs(rate_small / lattice_rate - 1) < 5e-6
    assert abs(rate_small / lattice_rate - 1) < 0.1 * abs(rate / lattice_rate - 1)


def _poiseuille(H_walls, ny, g, tau):
    """Closed-form steady profile for BGK + halfway bounce-back + the
    trapezoidal (Guo) force: u(y) = (g/2nu)(y - y1)(y2 - y) + g(16 L - 3)/(24 nu),
    L = (tau - 1/2)^2; zero slip at the known magic value L = 3/16."""
    y1, y2 = H_walls
    nu = (tau - 0.5) / 3
    lam = (tau - 0.5) ** 2
    y = np.arange(ny, dtype=float)
    return g / (2 * nu) * (y - y1) * (y2 - y) + g * (16 * lam - 3) / (24 * nu)


@pytest.mark.parametrize("lattice", [oracle.D2Q9, oracle.D3Q19, oracle.D3Q27])
@pytest.mark.parametrize("tau", [0.6, 0.9, 0.5 + math.sqrt(3 / 16), 1.5])
@pytest.mark.parametrize("walls", [oracle.SOLID_ENDS, oracle.WALLS_OUTSIDE])
def test_poiseuille_closed_form(lattice, tau, walls):
    """Pin P9: steady forced channel flow between halfway bounce-back walls."""
    H = 16
    g = 1e-6
    ny = H + 2 if walls == oracle.SOLID_ENDS else H
    y1, y2 = (0.5, H + 0.5) if walls == oracle.SOLID_ENDS else (-0.5, H - 0.5)
    s = oracle.Sim(lattice, 1, ny, 1, tau=tau, force=(g, 0, 0), bc=(0, walls, 0))
    fluid = s.geometry()
    s.init_equilibrium(np.ones((1, ny, 1)), np.zeros((3, 1, ny, 1)))
    nu = (tau - 0.5) / 3
    steps = int(math.log(1e13) / (nu * (math.pi / H) ** 2)) + 1
    s.step(steps)
    _, u = s.moments()
    ux = u[0, 0, :, 0]
    want = _poiseuille((y1, y2), ny, g, tau)
    fl = fluid[0, :, 0]
    assert np.abs(ux[fl] - want[fl]).max() / want[fl].max() < 1e-8
    assert np.abs(u[1]).max() < 1e-14  # roundoff of sum e_y f; u_x is ~1e-3


def test_adjoint_closed_form_mean_velocity():
    """Pin P12 (periodic): for J = sum_x u_x^N, dJ/du0_x = 1 everywhere,
    dJ/dF_x = V (N + 1/2)/rho0, dJ/dF_y = dJ/dF_z = 0 and dJ/dtau = 0,
    because the collision adds exactly F of momentum per node per step."""
    dims = (5, 4, 6)
    nx, ny, nz = dims
    rho, u, noise = _tg3(dims)
    ubar = np.zeros((3, nz, ny, nx))
    ubar[0] = 1.0
    N = 7
    u0bar, taubar, Fbar = oracle.adjoint(oracle.D3Q19, dims, 0.7, (1e-5, 0, 0), (0, 0, 0), rho, u,
                                         ubar, N, noise)
    V = nx * ny * nz
    assert np.abs(u0bar[0] - 1).max() < 1e-12
    assert np.abs(u0bar[1:]).max() < 1e-12
    assert abs(Fbar[0] / (V * (N + 0.5)) - 1) < 1e-12
    assert np.abs(Fbar[1:]).max() < 1e-10
    assert abs(taubar) < 1e-10


@pytest.mark.parametrize("lattice,dims,bc,opts", [
    (oracle.D2Q9, (6, 7, 1), (0, 0, 0), {}),
    (oracle.D2Q9, (5, 8, 1), (0, 1, 0), {}),
    (oracle.D3Q19, (4, 6, 5), (0, 1, 0), {}),
    (oracle.D3Q19, (5, 4, 4), (2, 0, 1), {}),
    (oracle.D3Q27, (4, 5, 4), (0, 1, 2), {}),
    (oracle.D2Q9, (6, 7, 1), (0, 0, 0), {"compressible": True}),
    (oracle.D3Q19, (5, 6, 4), (0, 1, 2), {"compressible": True}),
    (oracle.D2Q9, (5, 7, 1), (0, 3, 0), {}),
    (oracle.D3Q19, (4, 5, 6), (2, 0, 3), {}),
    (oracle.D3Q27, (5, 4, 4), (3, 1, 0), {"compressible": True}),
    (oracle.D3Q19, (7, 6, 5), (0, 3, 0), {"solid": "box"}),
])
def test_adjoint_matches_complex_step_tangent(lattice, dims, bc, opts):
    """Pin P13: the transposed run (complex-step Jacobians of each collision,
    transposed propagation) and the complex-step tangent of the whole forward
    run give the same directional derivative of J = 1/2 |u^N - u_tgt|^2 along
    random directions in (u0, tau, F); for both equilibria, halfway and nodal
    walls and a solid mask."""
    nx, ny, nz = dims
    D = 2 if lattice == oracle.D2Q9 else 3
    rng = np.random.default_rng(7)
    rho = 1.0 + 0.01 * rng.standard_normal((nz, ny, nx))
    u0 = np.zeros((3, nz, ny, nx))
    u0[:D] = 0.03 * rng.standard_normal((D, nz, ny, nx))
    u_tgt = np.zeros_like(u0)
    u_tgt[:D] = 0.03 * rng.standard_normal((D, nz, ny, nx))
    F = np.zeros(3)
    F[:D] = [2e-5, -1e-5, 3e-5][:D]
    Q = {oracle.D2Q9: 9, oracle.D3Q19: 19, oracle.D3Q27: 27}[lattice]
    noise = 1e-4 * rng.standard_normal((Q, nz, ny, nx))
    tau, N = 0.8, 9
    comp = opts.get("compressible", False)
    solid = _box_mask(dims, (2, 2, 1), (4, 3, 3)) if opts.get("solid") else None
    s = oracle.Sim(lattice, *dims, tau=tau, force=F, bc=bc, compressible=comp)
    if solid is not None:
        s.set_solid(solid)
    s.init_equilibrium(rho, u0, noise)
    s.step(N)
    _, uN = s.moments()
    fluid = s.geometry()
    u_tgt *= fluid
    ubar = (uN - u_tgt) * fluid
    ubar[D:] = 0.0
    u0bar, taubar, Fbar = oracle.adjoint(lattice, dims, tau, F, bc, rho, u0, ubar, N, noise,
                                         solid=solid, compressible=comp)
    for trial in range(3):
        du0 = np.zeros_like(u0)
        du0[:D] = rng.standard_normal((D, nz, ny, nx))
        dtau = rng.standard_normal()
        dF = np.zeros(3)
        dF[:D] = rng.standard_normal(D)
        J, dJ = oracle.cs_objective(lattice, dims, tau, F, bc, rho, u0, u_tgt, N, dtau=dtau,
                                    dforce=dF, du0=du0, noise=noise, solid=solid,
                                    compressible=comp)
        adj = (u0bar * du0).sum() + taubar * dtau + Fbar @ dF
        assert abs(adj - dJ) <= 1e-12 * abs(dJ), (adj, dJ)
        assert abs(J - 0.5 * (ubar ** 2).sum()) < 1e-14


def test_objective_finite_difference():
    """The complex-step directional derivative agrees with an FP64 central
    difference of the real forward run (P13's tangent is itself checked)."""
    dims = (4, 5, 3)
    nx, ny, nz = dims
    rng = np.random.default_rng(8)
    rho = np.ones((nz, ny, nx))
    u0 = 0.02 * rng.standard_normal((3, nz, ny, nx))
    u_tgt = 0.02 * rng.standard_normal((3, nz, ny, nx))
    du0 = rng.standard_normal((3, nz, ny, nx))
    F = (1e-5, 0, 0)
    _, dJ = oracle.cs_objective(oracle.D3Q19, dims, 0.7, F, (0, 0, 0), rho, u0, u_tgt, 6,
                                dtau=0.3, du0=du0)
    eps = 1e-6

    def J(sign):
        s = oracle.Sim(oracle.D3Q19, *dims, tau=0.7 + sign * eps * 0.3, force=F)
        s.init_equilibrium(rho, u0 + sign * eps * du0)
        s.step(6)
        return 0.5 * ((s.moments()[1] - u_tgt) ** 2).sum()

    fd = (J(1) - J(-1)) / (2 * eps)
    assert abs(fd - dJ) < 1e-7 * abs(dJ)


def _box_mask(dims, lo, hi):
    nx, ny, nz = dims
    m = np.zeros((nz, ny, nx), dtype=np.uint8)
    m[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] = 1
    return m


def test_solid_mask_equals_solid_end_planes():
    """A user mask marking the first and last y planes gives exactly the same
    run as the solid-ends boundary (SetGeometry with a geo array)."""
    dims = (6, 9, 5)
    nx, ny, nz = dims
    rho, u, noise = _tg3(dims)
    a = oracle.Sim(oracle.D3Q19, *dims, tau=0.8, force=(1e-5, 0, 0), bc=(0, 1, 0))
    b = oracle.Sim(oracle.D3Q19, *dims, tau=0.8, force=(1e-5, 0, 0))
    m = np.zeros((nz, ny, nx), dtype=np.uint8)
    m[:, 0, :] = m[:, -1, :] = 1
    b.set_solid(m)
    assert np.array_equal(a.geometry(), b.geometry())
    for s in (a, b):
        s.init_equilibrium(rho, u, noise)
        s.step(7)
    assert np.array_equal(a.get_populations(), b.get_populations())
    assert np.array_equal(a.wall_force(), b.wall_force())


@pytest.mark.parametrize("lattice", [oracle.D3Q19, oracle.D3Q27])
def test_pure_streaming_around_an_obstacle_is_a_permutation(lattice):
    dims = (7, 6, 5)
    Q = 19 if lattice == oracle.D3Q19 else 27
    s = oracle.Sim(lattice, *dims, tau=math.inf)
    s.set_solid(_box_mask(dims, (2, 2, 1), (4, 4, 3)))
    fluid = s.geometry()
    f0 = np.random.default_rng(3).uniform(0, 0.1, size=(Q,) + fluid.shape) * fluid
    s.set_populations(f0)
    s.step(3)
    f = s.get_populations()
    assert np.array_equal(np.sort(f[:, fluid].ravel()), np.sort(f0[:, fluid].ravel()))


@pytest.mark.parametrize("lattice", [oracle.D2Q9, oracle.D3Q19, oracle.D3Q27])
@pytest.mark.parametrize("walls", [oracle.SOLID_ENDS, oracle.WALLS_OUTSIDE])
def test_wall_force_balances_body_force_in_a_channel(lattice, walls):
    """Momentum balance (Sec. 4 momentum exchange): at steady state the walls
    take exactly the momentum the body force puts in, V_fluid * g per step."""
    ny, g, tau = 14, 1e-6, 0.8
    nz = 1 if lattice == oracle.D2Q9 else 2
    s = oracle.Sim(lattice, 3, ny, nz, tau=tau, force=(g, 0, 0), bc=(0, walls, 0))
    fluid = s.geometry()
    s.init_equilibrium(np.ones(fluid.shape), np.zeros((3,) + fluid.shape))
    H = ny - 2 if walls == oracle.SOLID_ENDS else ny
    s.step(int(math.log(1e12) / ((tau - 0.5) / 3 * (math.pi / H) ** 2)))
    F = s.wall_force()
    V = fluid.sum()
    assert abs(F[0] / (V * g) - 1) < 1e-9
    assert np.abs(F[1:]).max() < 1e-9 * V * g


@pytest.mark.parametrize("lattice", [oracle.D3Q19, oracle.D3Q27])
def test_wall_force_on_an_obstacle_balances_body_force(lattice):
    """A block obstacle in a periodic box driven by a body force: at steady
    state the drag on the obstacle, averaged over two consecutive
    propagations (the per-step force can carry a persistent period-2
    oscillation around obstacles), equals V_fluid * g."""
    dims = (8, 7, 6)
    g, tau = 1e-6, 0.9
    s = oracle.Sim(lattice, *dims, tau=tau, force=(g, 0, 0))
    s.set_solid(_box_mask(dims, (3, 2, 2), (5, 5, 4)))
    fluid = s.geometry()
    s.init_equilibrium(np.ones(fluid.shape), np.zeros((3,) + fluid.shape))
    s.step(6000)
    F1 = s.wall_force()
    s.step(1)
    F = 0.5 * (F1 + s.wall_force())
    V = fluid.sum()
    assert abs(F[0] / (V * g) - 1) < 1e-8
    assert np.abs(F[1:]).max() < 1e-8 * V * g
