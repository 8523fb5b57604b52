"""Whole-field FP64 parity at the workloads' own sizes and lengths, in the
launch configurations the benchmark times: every population of every node
and every velocity component against the CPU oracle run on the same seeded
inputs (the paper's CPU-only vs GPU comparison, Sec. 5), relative error
<= 1e-12 (max |gpu - oracle| / max |oracle|)."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2201_11330_amd import lbm
from paper_2201_11330_amd import workloads as W
from parity_utils import rel_err

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

TOL = 1e-12


def _compare(tag, sim, ref):
    """Whole-field e_f and e_u of the GPU context against the oracle; frees
    the GPU copies before the next field comes over."""
    f_or = ref.get_populations()
    f = sim.get_populations().cpu().numpy()
    ef = rel_err(f, f_or)
    del f, f_or
    _, u_or = ref.moments()
    _, u = sim.moments()
    eu = rel_err(u.cpu().numpy(), u_or)
    del u
    torch.cuda.empty_cache()
    print(f"{tag}: e_f {ef:.2e} e_u {eu:.2e}", flush=True)
    return ef, eu


def test_taylor_green_256_200_steps_whole_field():
    """Workload D3Q19 256^3 periodic FP64, 3D Taylor-Green U0 = 0.05 plus
    U(+-1e-6) population noise (seed 2), tau = 0.6, 200 steps, as lbm_step(1)
    launches of the two-nodes-per-work-item kernel (the benchmark's kernel
    and launch)."""
    n, tau, steps = 256, 0.6, 200
    rho, u = W.taylor_green_3d(n, U0=0.05)
    noise = W.population_noise(W.D3Q19, (n, n, n), 1e-6, seed=2)
    sim = lbm.LBM(lbm.D3Q19, n, n, n, tau)
    sim.init_equilibrium(rho, u, noise)
    for _ in range(steps):
        sim.step(1)
    ref = oracle.Sim(oracle.D3Q19, n, n, n, tau=tau)
    ref.init_equilibrium(rho, u, noise)
    del noise
    ref.step(steps)
    ef, eu = _compare("D3Q19 256^3 x 200", sim, ref)
    red, red_or = sim.reduce(), ref.reduce()
    sim.close()
    ref.close()
    assert ef <= TOL and eu <= TOL
    assert abs(red["mass"] / red_or["mass"] - 1) <= TOL
    assert abs(red["ke"] / red_or["ke"] - 1) <= 1e-10
    assert abs(red["umax"] / red_or["umax"] - 1) <= TOL


def test_channel_1000_steps_whole_field():
    """Workload D3Q19 channel 512 x 128 x 128 (x, z periodic; solid planes
    y = 0 and 127, halfway bounce-back), g_x = 1e-6, tau = 0.9, u ~ U(+-1e-4)
    (seed 3), 1000 steps in one lbm_step(1000) call."""
    dims = (512, 128, 128)
    bc = (W.PERIODIC, W.SOLID_ENDS, W.PERIODIC)
    tau, force, steps = 0.9, (1e-6, 0.0, 0.0), 1000
    rho, u = W.channel(*dims, amplitude=1e-4, seed=3, bc=bc)
    sim = lbm.LBM(lbm.D3Q19, *dims, tau, force=force, bc=bc)
    sim.init_equilibrium(rho, u)
    sim.step(steps)
    ref = oracle.Sim(oracle.D3Q19, *dims, tau=tau, force=force, bc=bc)
    ref.init_equilibrium(rho, u)
    ref.step(steps)
    ef, eu = _compare("channel 512x128x128 x 1000", sim, ref)
    sim.close()
    ref.close()
    assert ef <= TOL and eu <= TOL


def test_taylor_green_2d_128_1000_steps_one_call():
    """Workload D2Q9 128^2, tau = 0.8, 1000 steps as one lbm_step(1000) call:
    the four-steps-per-launch kernel on 16 x 16 regions (the benchmark's
    small_2d launch), whole field against the oracle."""
    n, tau, steps = 128, 0.8, 1000
    rho, u = W.taylor_green_2d(n, U0=0.01)
    sim = lbm.LBM(lbm.D2Q9, n, n, 1, tau)
    sim.init_equilibrium(rho, u)
    sim.step(steps)
    assert sim.steps_taken == steps
    ref = oracle.Sim(oracle.D2Q9, n, n, 1, tau=tau)
    ref.init_equilibrium(rho, u)
    ref.step(steps)
    ef, eu = _compare("D2Q9 128^2 x 1000 (one call)", sim, ref)
    red, red_or = sim.reduce(), ref.reduce()
    sim.close()
    ref.close()
    assert ef <= TOL and eu <= TOL
    assert abs(red["ke"] / red_or["ke"] - 1) <= 1e-10


def test_d2q9_4096_four_step_launches_whole_field():
    """D2Q9 4096^2 periodic Taylor-Green, tau = 0.8, 8 steps in one call: two
    four-step launches streamed up strips of 224 columns (the benchmark's
    large_2d launch, segments of 103 rows with a ragged last one), whole
    field against the oracle."""
    n, tau, steps = 4096, 0.8, 8
    rho, u = W.taylor_green_2d(n, U0=0.01)
    noise = W.population_noise(W.D2Q9, (n, n, 1), 1e-6, seed=40)
    sim = lbm.LBM(lbm.D2Q9, n, n, 1, tau)
    sim.init_equilibrium(rho, u, noise)
    sim.step(steps)
    ref = oracle.Sim(oracle.D2Q9, n, n, 1, tau=tau)
    ref.init_equilibrium(rho, u, noise)
    ref.step(steps)
    ef, eu = _compare("D2Q9 4096^2 x 8 (streamed strips)", sim, ref)
    sim.close()
    ref.close()
    assert ef <= TOL and eu <= TOL


def test_taylor_green_128_500_steps_whole_field():
    """D3Q19 128^3 periodic Taylor-Green U0 = 0.05 plus U(+-1e-6) noise,
    tau = 0.6, 500 steps in one call: the FP64 run of the reduced-precision
    workload at a size the oracle finishes, whole field."""
    n, tau, steps = 128, 0.6, 500
    rho, u = W.taylor_green_3d(n, U0=0.05)
    noise = W.population_noise(W.D3Q19, (n, n, n), 1e-6, seed=4)
    sim = lbm.LBM(lbm.D3Q19, n, n, n, tau)
    sim.init_equilibrium(rho, u, noise)
    sim.step(steps)
    ref = oracle.Sim(oracle.D3Q19, n, n, n, tau=tau)
    ref.init_equilibrium(rho, u, noise)
    ref.step(steps)
    ef, eu = _compare("D3Q19 128^3 x 500", sim, ref)
    sim.close()
    ref.close()
    assert ef <= TOL and eu <= TOL
