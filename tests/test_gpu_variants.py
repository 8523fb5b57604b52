"""GPU parity of the two model variants against the oracle: the weakly
compressible equilibrium of Eq. (feq) and the walls of the modified nodal
bounce-back (Sec. 2.2), alone and combined with solid masks, in both
propagation patterns, the reduced-precision storages, the monitor, the wall
force and the discrete adjoint."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2201_11330_amd import lbm
from paper_2201_11330_amd import workloads as W
from parity_utils import quantize, rel_err, run_gpu, run_oracle, ulp

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _inputs(lattice, dims, seed, drho=0.1, U=0.04, noise=1e-4):
    """Densities far from 1 (where the two equilibria differ), random
    velocities and population noise."""
    nx, ny, nz = dims
    rng = np.random.default_rng(seed)
    rho = 1.0 + drho * rng.uniform(-1.0, 1.0, (nz, ny, nx))
    u = U * rng.standard_normal((3, nz, ny, nx))
    if lattice == W.D2Q9:
        u[2] = 0.0
    n = noise * rng.standard_normal((W.Q_OF[lattice], nz, ny, nx))
    return rho, u, n


def _mask(dims, on):
    if not on:
        return None
    nx, ny, nz = dims
    c = ((nx - 1) / 2 + 0.3, (ny - 1) / 2 - 0.2, max((nz - 1) / 2 + 0.1, 0.0))
    return W.sphere_mask(dims, c, min(2.2, (min(nx, ny) - 3) / 2))


# (lattice, dims, bc, force, compressible, mask)
CASES = [
    (W.D2Q9, (33, 17, 1), (0, 0, 0), (1e-5, -2e-5, 0), True, False),
    (W.D3Q19, (19, 14, 11), (0, 1, 2), (1e-5, 0, 2e-5), True, False),
    (W.D3Q27, (13, 9, 10), (2, 0, 0), (0, 1e-5, 0), True, True),
    (W.D2Q9, (21, 15, 1), (0, 3, 0), (1e-5, 0, 0), False, False),
    (W.D3Q19, (17, 12, 9), (1, 0, 3), (1e-5, 2e-5, 0), False, False),
    (W.D3Q27, (10, 11, 9), (3, 2, 0), (0, 1e-5, -1e-5), False, True),
    # several 4096-node tiles and a ragged last tile
    (W.D3Q19, (300, 7, 5), (0, 3, 0), (1e-5, 0, 0), True, True),
]


def _cid(c):
    return (f"Q{W.Q_OF[c[0]]}-{'x'.join(map(str, c[1]))}-bc{''.join(map(str, c[2]))}"
            f"{'-comp' if c[4] else ''}{'-mask' if c[5] else ''}")


@pytest.mark.parametrize("aa", [False, True], ids=["AB", "AA"])
@pytest.mark.parametrize("case", CASES, ids=_cid)
def test_fp64_parity(case, aa):
    lattice, dims, bc, force, comp, mk = case
    solid = _mask(dims, mk)
    rho, u, noise = _inputs(lattice, dims, seed=5)
    steps = 9
    print(f"case {_cid(case)} aa={aa}", flush=True)
    f_or, r_or, u_or, red_or = run_oracle(lattice, dims, 0.7, force, bc, rho, u, noise, steps,
                                          solid=solid, compressible=comp)
    f, r, v, red = run_gpu(lattice, dims, 0.7, force, bc, rho, u, noise, steps, aa=aa,
                           solid=solid, compressible=comp)
    ef, er, eu = rel_err(f, f_or), rel_err(r, r_or), rel_err(v, u_or)
    print(f"  f {ef:.2e} rho {er:.2e} u {eu:.2e}")
    assert ef <= TOL and er <= TOL and eu <= TOL
    assert abs(red["mass"] - red_or["mass"]) <= TOL * abs(red_or["mass"])
    assert abs(red["ke"] - red_or["ke"]) <= 1e-11 * red_or["ke"]
    assert abs(red["umax"] - red_or["umax"]) <= TOL * red_or["umax"]


def test_compressible_and_incompressible_differ_on_the_gpu():
    """Control: at densities far from 1 the two models give different
    states, so the parity above distinguishes them."""
    lattice, dims = W.D3Q19, (9, 8, 7)
    rho, u, noise = _inputs(lattice, dims, seed=6)
    a = run_gpu(lattice, dims, 0.7, (1e-5, 0, 0), (0, 0, 0), rho, u, noise, 3)[0]
    b = run_gpu(lattice, dims, 0.7, (1e-5, 0, 0), (0, 0, 0), rho, u, noise, 3, compressible=True)[0]
    assert rel_err(a, b) > 1e-4


@pytest.mark.parametrize("aa", [False, True], ids=["AB", "AA"])
def test_nodal_state_roundtrip_follows_eq_bb(aa):
    """lbm_set_populations / lbm_get_populations with nodal walls: the
    unknown populations of wall nodes read back as the opposite ones (what
    the oracle keeps), everything else bit-exact."""
    lattice, dims, bc = W.D3Q19, (11, 9, 8), (0, 3, 1)
    rng = np.random.default_rng(12)
    _, t = oracle.lattice_tables(lattice)
    f = t[:, None, None, None] * (1.0 + 0.01 * rng.standard_normal((19, 8, 9, 11)))
    ref = oracle.Sim(lattice, *dims, tau=0.7, bc=bc)
    ref.set_populations(f)
    want = ref.get_populations()
    sim = lbm.LBM(lattice, *dims, 0.7, bc=bc, aa=aa)
    sim.set_populations(f)
    got = sim.get_populations().cpu().numpy()
    assert np.array_equal(got, want)
    assert not np.array_equal(want, f * ref.geometry())  # the rule changed some values
    ref.step(3)
    sim.step(3)
    assert rel_err(sim.get_populations().cpu().numpy(), ref.get_populations()) <= TOL


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16", "e4m11"])
@pytest.mark.parametrize("aa", [False, True], ids=["AB", "AA"])
def test_reduced_precision_one_step(storage, aa):
    """Deviation storage with both variants on (compressible, nodal walls
    across y): from a state exactly representable in the storage format one
    step equals the FP64 oracle's step rounded to the format, within one
    unit in the last place plus FP32 arithmetic error."""
    lattice, dims, bc, force, tau = W.D3Q19, (37, 21, 10), (0, 3, 0), (1e-5, 0, 0), 0.7
    rho, u, noise = _inputs(lattice, dims, seed=9, drho=0.05, noise=1e-4)
    ref = oracle.Sim(lattice, *dims, tau=tau, force=force, bc=bc, compressible=True)
    ref.init_equilibrium(rho, u, noise)
    _, t = oracle.lattice_tables(lattice)
    tw = t[:, None, None, None] * np.ones((1,) + rho.shape)
    g0 = quantize(ref.get_populations() - tw, storage)
    g0[np.abs(g0) < 1e-8] = 0.0
    f0 = g0 + tw
    ref.set_populations(f0)
    sim = lbm.LBM(lattice, *dims, tau, force=force, bc=bc, storage=storage, aa=aa,
                  compressible=True)
    sim.set_populations(f0)
    assert np.array_equal(sim.get_populations().cpu().numpy() - tw, g0)
    ref.step(1)
    sim.step(1)
    g_ref = ref.get_populations() - tw
    g = sim.get_populations().cpu().numpy() - tw
    tol = ulp(g_ref, storage) + 64 * np.finfo(np.float32).eps * np.abs(g_ref).max()
    worst = (np.abs(g - g_ref) / tol).max()
    print(f"{storage} aa={aa}: worst error / tolerance = {worst:.3f}")
    assert worst <= 1.0


def test_nodal_poiseuille_closed_form_on_the_gpu():
    """Steady channel between nodal walls: u(y) = (g/2nu) y (H - y) +
    (2 tau + 1/2) g (the closed form pinned against the oracle), on a 3D box
    with the FP64 two-lattice kernel."""
    H, g, tau = 16, 1e-6, 0.9
    dims = (8, H + 1, 4)
    sim = lbm.LBM(W.D3Q19, *dims, tau, force=(g, 0, 0), bc=(0, 3, 0), graph=True)
    sim.init_equilibrium(np.ones(dims[::-1]), np.zeros((3,) + dims[::-1]))
    nu = (tau - 0.5) / 3
    sim.step(int(math.log(1e13) / (nu * (math.pi / H) ** 2)) + 1)
    _, u = sim.moments()
    prof = u[0].cpu().numpy()
    y = np.arange(H + 1, dtype=float)
    want = g / (2 * nu) * y * (H - y) + (2 * tau + 0.5) * g
    err = np.abs(prof - want[None, :, None]).max() / want.max()
    print(f"nodal Poiseuille: {err:.2e}")
    assert err < 1e-8


def test_compressible_channel_velocity_is_force_over_density():
    """Compressible model at rho = 1.5 driven by F = 1.5 g: the halfway
    Poiseuille profile of the acceleration g."""
    H, g, tau, rho0 = 16, 1e-6, 0.9, 1.5
    dims = (4, H + 2, 4)
    sim = lbm.LBM(W.D3Q19, *dims, tau, force=(rho0 * g, 0, 0), bc=(0, 1, 0), compressible=True,
                  graph=True)
    sim.init_equilibrium(np.full(dims[::-1], rho0), np.zeros((3,) + dims[::-1]))
    nu = (tau - 0.5) / 3
    sim.step(int(math.log(1e13) / (nu * (math.pi / H) ** 2)) + 1)
    r, u = sim.moments()
    y = np.arange(H + 2, dtype=float)
    want = (g / (2 * nu) * (y - 0.5) * (H + 0.5 - y)
            + g * (16 * (tau - 0.5) ** 2 - 3) / (24 * nu))[1:-1]
    prof = u[0].cpu().numpy()[:, 1:-1, :]
    err = np.abs(prof - want[None, :, None]).max() / want.max()
    print(f"compressible channel at rho {rho0}: {err:.2e}")
    assert err < 1e-8
    assert np.abs(r.cpu().numpy()[:, 1:-1, :] - rho0).max() < 1e-12


def test_wall_force_with_nodal_walls_counts_the_mask_only():
    """Momentum exchange on a sphere in a channel with nodal walls: GPU vs
    oracle, the nodal wall links excluded on both sides."""
    lattice, dims, bc = W.D3Q19, (16, 13, 10), (0, 3, 0)
    solid = W.sphere_mask(dims, (7.5, 6.2, 4.6), 2.4)
    rho, u, noise = _inputs(lattice, dims, seed=17, drho=0.01)
    ref = oracle.Sim(lattice, *dims, tau=0.8, force=(1e-5, 0, 0), bc=bc)
    ref.set_solid(solid)
    ref.init_equilibrium(rho, u * ref.geometry(), noise)
    ref.step(6)
    F_or = np.asarray(ref.wall_force())
    sim = lbm.LBM(lattice, *dims, 0.8, force=(1e-5, 0, 0), bc=bc)
    sim.set_solid(solid)
    sim.init_equilibrium(rho, u * ref.geometry(), noise)
    sim.step(6)
    F = np.asarray(sim.wall_force())
    print(f"wall force {F} oracle {F_or}")
    assert np.abs(F - F_or).max() <= 1e-12 * np.abs(F_or).max()


ADJ_CASES = [
    # (lattice, dims, bc, force, compressible, mask, n, k)
    (W.D3Q19, (9, 7, 6), (0, 0, 0), (1e-5, -2e-5, 3e-5), True, False, 12, 4),
    (W.D2Q9, (11, 9, 1), (0, 1, 0), (1e-5, 2e-5, 0), True, False, 10, 10),
    (W.D3Q19, (8, 10, 7), (0, 3, 0), (2e-5, 0, 0), False, False, 10, 5),
    (W.D2Q9, (9, 12, 1), (3, 0, 0), (0, 1e-5, 0), False, False, 8, 1),
    (W.D3Q27, (9, 8, 7), (2, 0, 3), (1e-5, 1e-5, 0), True, True, 9, 3),
    (W.D3Q19, (12, 10, 9), (0, 3, 0), (1e-5, 0, 0), True, True, 10, 5),
]


@pytest.mark.parametrize("case", ADJ_CASES, ids=lambda c: _cid(c[:6]) + f"-n{c[6]}k{c[7]}")
def test_adjoint_matches_oracle(case):
    """Closed-form GPU adjoint (compressible Jacobian, transposed Eq. (bb)
    on nodal walls, masks) vs the oracle's complex-step adjoint (FP64)."""
    lattice, dims, bc, force, comp, mk, n, k = case
    tau = 0.7
    nx, ny, nz = dims
    D = 2 if lattice == W.D2Q9 else 3
    solid = _mask(dims, mk)
    rho, u0, noise = _inputs(lattice, dims, seed=21, drho=0.05, U=0.03)
    rng = np.random.default_rng(22)
    s = oracle.Sim(lattice, *dims, tau=tau, force=force, bc=bc, compressible=comp)
    if solid is not None:
        s.set_solid(solid)
    fluid = s.geometry()
    u0 = u0 * fluid
    s.init_equilibrium(rho, u0, noise)
    s.step(n)
    _, uN = s.moments()
    u_tgt = 0.03 * rng.standard_normal(u0.shape) * fluid
    ubar = (uN - u_tgt) * fluid
    ubar[D:] = 0.0
    ob_u0, ob_tau, ob_F = oracle.adjoint(lattice, dims, tau, force, bc, rho, u0, ubar, n, noise,
                                         solid=solid, compressible=comp)
    sim = lbm.LBM(lattice, *dims, tau, force=force, bc=bc, compressible=comp)
    if solid is not None:
        sim.set_solid(solid)
    sim.init_equilibrium(rho, u0, noise)
    ckpt = sim.forward_record(n, k)
    gb_u0, gb_tau, gb_F = sim.adjoint(n, k, ckpt, u0, ubar, rho0=rho)
    gb_u0 = gb_u0.cpu().numpy()
    e_u0 = np.abs(gb_u0 - ob_u0).max() / np.abs(ob_u0).max()
    scale = np.abs(ob_u0).sum()
    e_tau = abs(gb_tau - ob_tau) / scale
    e_F = np.abs(np.asarray(gb_F) - ob_F).max() / scale
    print(f"{_cid(case[:6])}: u0bar {e_u0:.2e} taubar {e_tau:.2e} Fbar {e_F:.2e}")
    assert e_u0 <= TOL and e_tau <= TOL and e_F <= TOL


def test_compressible_adjoint_rejects_n_zero_and_missing_rho0():
    sim = lbm.LBM(W.D3Q19, 6, 5, 4, 0.7, compressible=True)
    sim.init_equilibrium(np.ones((4, 5, 6)), np.zeros((3, 4, 5, 6)))
    ckpt = sim.forward_record(2, 1)
    z = np.zeros((3, 4, 5, 6))
    with pytest.raises(lbm.LBMError):
        sim.adjoint(0, 1, ckpt, z, z, rho0=np.ones((4, 5, 6)))
    with pytest.raises(lbm.LBMError):
        sim.adjoint(2, 1, ckpt, z, z)
    sim.adjoint(2, 1, ckpt, z, z, rho0=np.ones((4, 5, 6)))


def test_autograd_rollout_with_compressible_model_and_nodal_walls():
    """LBMRollout (torch.autograd.Function over lbm_forward_record and
    lbm_adjoint) for the compressible model in a channel with nodal walls:
    the gradients of J = 1/2 |u^n - u_tgt|^2 with respect to u0, tau and F
    equal the oracle's complex-step adjoint."""
    lattice, dims, bc = W.D3Q19, (10, 9, 6), (0, 3, 0)
    nx, ny, nz = dims
    tau, F, n, k = 0.75, (2e-5, 0.0, -1e-5), 8, 4
    rho, u0, noise = _inputs(lattice, dims, seed=41, drho=0.05, U=0.03, noise=0.0)
    rng = np.random.default_rng(42)
    u_tgt = 0.03 * rng.standard_normal(u0.shape)
    u0t = torch.tensor(u0, device="cuda", requires_grad=True)
    taut = torch.tensor(tau, dtype=torch.float64, requires_grad=True)
    Ft = torch.tensor(F, dtype=torch.float64, requires_grad=True)
    uN = lbm.LBMRollout.apply(u0t, taut, Ft, rho, n, k, lattice, bc, "f64", None, True)
    J = 0.5 * ((uN - torch.tensor(u_tgt, device="cuda")) ** 2).sum()
    J.backward()
    s = oracle.Sim(lattice, *dims, tau=tau, force=F, bc=bc, compressible=True)
    s.init_equilibrium(rho, u0)
    s.step(n)
    ubar = s.moments()[1] - u_tgt
    ob_u0, ob_tau, ob_F = oracle.adjoint(lattice, dims, tau, F, bc, rho, u0, ubar, n,
                                         compressible=True)
    e_u0 = np.abs(u0t.grad.cpu().numpy() - ob_u0).max() / np.abs(ob_u0).max()
    scale = np.abs(ob_u0).sum()
    e_tau = abs(taut.grad.item() - ob_tau) / scale
    e_F = np.abs(Ft.grad.numpy() - ob_F).max() / scale
    print(f"autograd compressible + nodal: u0 {e_u0:.2e} tau {e_tau:.2e} F {e_F:.2e}")
    assert e_u0 <= TOL and e_tau <= TOL and e_F <= TOL
