"""Full workloads on the GPU: the forced channel against the Poiseuille
closed form and a 1-column oracle run, and the 512^3 reduced-precision
Taylor-Green runs against the FP64 run on the same seed."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2201_11330_amd import lbm
from paper_2201_11330_amd import workloads as W

pytestmark = pytest.mark.gpu


def _poiseuille(y1, y2, ny, g, tau):
    """Steady profile between halfway bounce-back walls with BGK and the
    trapezoidal force: (g/2nu)(y - y1)(y2 - y) + g(16 L - 3)/(24 nu)."""
    nu = (tau - 0.5) / 3
    lam = (tau - 0.5) ** 2
    y = np.arange(ny, dtype=float)
    return g / (2 * nu) * (y - y1) * (y2 - y) + g * (16 * lam - 3) / (24 * nu)


@pytest.mark.parametrize("walls", [W.SOLID_ENDS, W.WALLS_OUTSIDE])
@pytest.mark.parametrize("aa", [False, True], ids=["AB", "AA"])
def test_poiseuille_steady_3d(walls, aa):
    """A 3D D3Q19 channel run to steady state reproduces the closed form at
    every node (x-z uniform) to 1e-8 of the centreline velocity."""
    nx, ny, nz, tau, g = 24, 32, 16, 0.9, 1e-6
    bc = (W.PERIODIC, walls, W.PERIODIC)
    H = ny - 2 if walls == W.SOLID_ENDS else ny
    y1, y2 = (0.5, ny - 1.5) if walls == W.SOLID_ENDS else (-0.5, ny - 0.5)
    nu = (tau - 0.5) / 3
    steps = 2 * int(math.log(1e11) / (nu * (math.pi / H) ** 2) / 2) + 2
    sim = lbm.LBM(lbm.D3Q19, nx, ny, nz, tau, force=(g, 0, 0), bc=bc, aa=aa)
    sim.init_equilibrium(np.ones((nz, ny, nx)), np.zeros((3, nz, ny, nx)))
    sim.step(steps)
    _, u = sim.moments()
    u = u.cpu().numpy()
    want = _poiseuille(y1, y2, ny, g, tau)
    fluid = np.ones(ny, bool)
    if walls == W.SOLID_ENDS:
        fluid[[0, -1]] = False
    err = np.abs(u[0][:, fluid, :] - want[None, fluid, None]).max() / want.max()
    print(f"steady channel walls={walls} aa={aa} steps={steps}: rel err {err:.2e}")
    assert err < 1e-8
    assert np.abs(u[1:]).max() < 1e-11 * want.max()  # roundoff of sum e_y f


@pytest.mark.slow
@pytest.mark.parametrize("walls", [W.SOLID_ENDS, W.WALLS_NODAL], ids=["halfway", "nodal"])
def test_channel_full_height_steady_state(walls):
    """The channel workload's height (128 nodes across y, g_x = 1e-6,
    tau = 0.9) run to steady state on a narrow periodic box: 250,000 steps,
    after which the slowest mode has decayed to exp(-nu (pi/H)^2 t) ~ 1e-9.
    The profile equals the closed form of the wall type (halfway: walls at
    0.5 and 126.5; nodal: walls on the nodes 0 and 127)."""
    nx, ny, nz, tau, g = 4, 128, 4, 0.9, 1e-6
    nu = (tau - 0.5) / 3
    sim = lbm.LBM(lbm.D3Q19, nx, ny, nz, tau, force=(g, 0, 0), bc=(0, walls, 0), graph=True)
    sim.init_equilibrium(np.ones((nz, ny, nx)), np.zeros((3, nz, ny, nx)))
    y = np.arange(ny, dtype=float)
    if walls == W.SOLID_ENDS:
        H, fl = ny - 2, slice(1, ny - 1)
        want = g / (2 * nu) * (y - 0.5) * (ny - 1.5 - y) + g * (16 * (tau - 0.5) ** 2 - 3) / (24 * nu)
    else:
        H, fl = ny - 1, slice(0, ny)
        want = g / (2 * nu) * y * (H - y) + (2 * tau + 0.5) * g
    steps = 250_000
    for k in range(5):
        sim.step(steps // 5)
        print(f"step {(k + 1) * steps // 5}", flush=True)
    _, u = sim.moments()
    prof = u[0].cpu().numpy()[:, fl, :]
    err = np.abs(prof - want[None, fl, None]).max() / want[fl].max()
    print(f"full-height channel ({'halfway' if walls == W.SOLID_ENDS else 'nodal'}): "
          f"{err:.2e} (transient {math.exp(-nu * (math.pi / H) ** 2 * steps):.1e})")
    assert err < 1e-8


def test_channel_workload_20000_steps():
    """Workload D3Q19 512 x 128 x 128 channel, g_x = 1e-6, tau = 0.9, 20000
    steps: the x-z averaged u_x(y) equals a 1-column oracle run (same walls,
    started from the plane-averaged initial velocity) up to the Reynolds
    stress of the 1e-4 perturbation.  Mass drifts only by the rounding of the
    FP64 weights: their exact sum is 1 - 2^-54, so every collision scales the
    mass by 1 + omega (sum w - 1) and n steps by n omega (sum w - 1)."""
    nx, ny, nz, tau, g, steps = 512, 128, 128, 0.9, 1e-6, 20000
    bc = (W.PERIODIC, W.SOLID_ENDS, W.PERIODIC)
    rho, u = W.channel(nx, ny, nz, amplitude=1e-4, seed=3, bc=bc)
    sim = lbm.LBM(lbm.D3Q19, nx, ny, nz, tau, force=(g, 0, 0), bc=bc)
    sim.init_equilibrium(rho, u)
    m0 = sim.reduce()["mass"]
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(sim.stream)
    sim.step(steps)
    e1.record(sim.stream)
    red = sim.reduce()
    ms = e0.elapsed_time(e1)
    mlups = nx * ny * nz * steps / (ms * 1e-3) / 1e6
    fluid_mlups = mlups * (ny - 2) / ny
    _, ug = sim.moments()
    prof = ug[0].mean(dim=(0, 2)).cpu().numpy()
    sim.close()
    # 1-column oracle run from the plane-averaged start
    ubar = u.mean(axis=(1, 3))  # [3][ny]
    u1 = np.zeros((3, 1, ny, 1))
    u1[:, 0, :, 0] = ubar
    col = oracle.Sim(oracle.D3Q19, 1, ny, 1, tau=tau, force=(g, 0, 0), bc=bc)
    col.init_equilibrium(np.ones((1, ny, 1)), u1)
    col.step(steps)
    _, uc = col.moments()
    ref = uc[0, 0, :, 0]
    err = np.abs(prof[1:-1] - ref[1:-1]).max() / ref.max()
    steady = _poiseuille(0.5, ny - 1.5, ny, g, tau)
    print(f"channel 20000 steps: {mlups:.0f} MLUPS ({fluid_mlups:.0f} fluid), centreline "
          f"{prof[ny // 2]:.6e} (steady {steady[ny // 2]:.6e}), vs 1-column {err:.2e}, "
          f"mass drift {abs(red['mass'] - m0) / m0:.1e}")
    assert err < 1e-5
    from fractions import Fraction
    wsum = sum(Fraction(x) for x in [1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    predicted = steps * (1 / tau) * float(wsum - 1)
    drift = (red["mass"] - m0) / m0
    assert abs(drift - predicted) < 1e-14, (drift, predicted)
    assert 0.5 < prof[ny // 2] / steady[ny // 2] < 1.0


def _tg_run(n, storage, steps, every, inputs, tau=0.6):
    rho, u, noise = inputs
    sim = lbm.LBM(lbm.D3Q19, n, n, n, tau, storage=storage)
    sim.init_equilibrium(rho, u, noise)
    ts, ke = [], []
    torch.cuda.synchronize()
    for it in range(0, steps + 1, every):
        ts.append(it)
        ke.append(sim.reduce()["ke"])
        if it < steps:
            sim.step(every)
    _, uN = sim.moments(dtype=torch.float32 if storage != "f64" else torch.float64)
    sim.close()
    return np.array(ts, float), np.array(ke), uN.to(torch.float64)


def _rate(ts, ke, skip=100):
    m = ts >= skip
    return -np.polyfit(ts[m], np.log(ke[m]), 1)[0]


# Measured on MI355X (this workload, these inputs): max |u - u_f64| / U0 and
# the relative KE decay-rate error of each storage.
MEASURED_512 = {"f32": (9.7e-6, 1.0e-3), "f16": (2.24e-3, 5.8e-2), "bf16": (2.64e-2, 0.251),
                "e4m11": (7.13e-4, 1.50e-2)}


@pytest.mark.slow
def test_reduced_precision_taylor_green_512():
    """Workload D3Q19 512^3 Taylor-Green, tau = 0.6, 500 steps: FP32, FP16,
    e4m11 and BF16 storage of f - w (FP32 arithmetic) against the FP64 run on the same
    inputs (population noise U(+-1e-6) from torch's device generator, seed 4,
    as in the benchmark's precision line).  Reported: max |u| error
    (absolute and / U0) and the relative error of the kinetic-energy decay
    rate (KE drops only ~1.5 % over the run, so a 1e-5 relative KE error is
    ~1e-3 of the rate).  There is no closed form (parity unpinned beyond the
    FP64 run, which the parity tests pin); each error is bounded at 3x its
    measured value, so a regression of that size fails."""
    n, steps, every, U0 = 512, 500, 10, 0.05
    rho, u0 = W.taylor_green_3d(n, U0=U0)
    noise = W.uniform_noise_device((19, n, n, n), 1e-6, seed=4)
    inputs = (torch.from_numpy(np.array(rho, copy=True)).cuda(),
              torch.from_numpy(np.array(u0, copy=True)).cuda(), noise)
    ts, ke64, u64 = _tg_run(n, "f64", steps, every, inputs)
    r64 = _rate(ts, ke64)
    for storage in ("f32", "f16", "bf16", "e4m11"):
        ts, ke, u = _tg_run(n, storage, steps, every, inputs)
        du = (u - u64).abs().max().item()
        rerr = abs(_rate(ts, ke) / r64 - 1)
        print(f"{storage}: max|u - u_f64| = {du:.3e} ({du / U0:.3e} of U0), "
              f"KE decay rate error {rerr:.3e} (FP64 rate {r64:.6e}/step)")
        del u
        torch.cuda.empty_cache()
        m_du, m_rate = MEASURED_512[storage]
        assert du / U0 < 3 * m_du and rerr < 3 * m_rate


@pytest.mark.slow
def test_maximum_size_box_sampled():
    """Largest box the 32-bit node index admits at this size class:
    1280^3 = 2.1e9 nodes (< 2^31), D3Q19 FP16 storage with the in-place AA
    pattern (80 GB; element offsets up to 4e10, beyond 2^32).  Random
    velocities (U(+-0.02) per component per node, so a wrong neighbour index
    shows as an O(0.02) error, far above FP16 rounding), two steps (one even,
    one odd), then u at sampled nodes -- corners and seams included -- against
    the oracle on each node's dependency window."""
    n, steps, tau = 1280, 2, 0.7
    N = n ** 3
    assert N < 2 ** 31
    sim = lbm.LBM(lbm.D3Q19, n, n, n, tau, storage="f16", aa=True)
    rho = torch.ones((n, n, n), dtype=torch.float64, device="cuda")
    u = W.uniform_noise_device((3, n, n, n), 0.02, seed=13)
    sim.init_equilibrium(rho, u)
    centers = [(0, 0, 0), (n - 1, n - 1, n - 1), (0, n - 1, 0), (n - 1, 0, n - 1),
               (640, 640, 640), (1, 1279, 1278), (1023, 511, 1279)]
    windows = []
    for (cx, cy, cz) in centers:
        ix = [(cx + d) % n for d in range(-steps, steps + 1)]
        iy = [(cy + d) % n for d in range(-steps, steps + 1)]
        iz = [(cz + d) % n for d in range(-steps, steps + 1)]
        ti = lambda v: torch.tensor(v, device="cuda")
        uw = u[:, ti(iz)][:, :, ti(iy)][:, :, :, ti(ix)].cpu().numpy()
        windows.append(uw)
    sim._keep = None
    del rho, u
    torch.cuda.empty_cache()
    sim.step(steps)
    red = sim.reduce()
    assert not red["unstable"]
    _, ug = sim.moments(dtype=torch.float32)
    worst = 0.0
    for (cx, cy, cz), uw in zip(centers, windows):
        w = 2 * steps + 1
        ref = oracle.Sim(oracle.D3Q19, w, w, w, tau=tau)
        ref.init_equilibrium(np.ones((w, w, w)), uw)
        ref.step(steps)
        _, ur = ref.moments()
        got = ug[:, cz, cy, cx].double().cpu().numpy()
        worst = max(worst, np.abs(got - ur[:, steps, steps, steps]).max())
    print(f"1280^3 FP16 AA: worst |u - u_oracle| at sampled nodes {worst:.2e}, "
          f"mass {red['mass']:.6e} (N = {N})")
    assert worst < 2e-4  # FP16 rounding of f - w is ~1e-5 here; an index error is ~2e-2
    assert abs(red["mass"] / N - 1) < 1e-6
