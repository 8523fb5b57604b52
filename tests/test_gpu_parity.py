"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle on the
same seeded inputs.  FP64 bar: relative error <= 1e-12 after N steps
(max |f_gpu - f_oracle| / max |f_oracle|, and the same for u), the paper's
own CPU-vs-GPU methodology (Sec. 5).  Permutation-only work (pure
streaming, state import/export, AA vs AB, translation) is compared bit for
bit."""
import math

import numpy as np
import pytest
import torch

from paper_2201_11330_amd import lbm
from paper_2201_11330_amd import workloads as W
from parity_utils import (inputs, quantize, rel_err, run_gpu, run_oracle, sampled_window_check,
                          ulp)

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _case_id(c):
    return "x".join(map(str, c[1])) + f"-bc{''.join(map(str, c[3]))}"


CASES_3D = [
    # lattice, dims, tau, bc, force, steps, input kind
    (W.D3Q19, (37, 29, 23), 0.6, (0, 0, 0), (0, 0, 0), 20, "tg"),
    (W.D3Q19, (300, 7, 5), 0.7, (0, 0, 0), (2e-6, -1e-6, 1e-6), 12, "tg"),
    # rows of 2 and 3 workgroups placed on one XCD each (ny a multiple of 8)
    (W.D3Q19, (300, 8, 5), 0.7, (0, 1, 0), (1e-5, 0, 0), 12, "channel"),
    (W.D3Q19, (530, 8, 3), 0.7, (0, 0, 0), (2e-6, -1e-6, 1e-6), 10, "tg"),
    (W.D3Q19, (257, 16, 2), 0.8, (0, 0, 0), (1e-5, 0, 0), 8, "tg"),  # second workgroup 1/256 busy
    (W.D3Q19, (40, 20, 18), 0.9, (0, 1, 0), (1e-5, 0, 0), 30, "channel"),
    (W.D3Q19, (33, 17, 12), 0.75, (2, 1, 2), (1e-5, 2e-6, -3e-6), 25, "channel"),
    (W.D3Q19, (1, 34, 1), 0.9, (0, 1, 0), (1e-5, 0, 0), 60, "channel"),
    (W.D3Q19, (5, 3, 4), 0.8, (0, 1, 0), (1e-5, 0, 1e-6), 9, "channel"),
    (W.D3Q19, (1, 1, 1), 0.8, (0, 0, 0), (1e-5, 0, 0), 5, "channel"),
    (W.D3Q19, (9, 11, 13), 0.55, (1, 1, 1), (1e-5, -1e-5, 1e-5), 15, "channel"),
    (W.D2Q9, (70, 33, 1), 0.8, (0, 1, 0), (1e-5, 0, 0), 40, "channel"),
    (W.D2Q9, (300, 45, 1), 1.2, (2, 0, 0), (0, 1e-5, 0), 30, "channel"),
    (W.D2Q9, (600, 16, 1), 0.8, (2, 0, 0), (0, 1e-5, 0), 20, "channel"),
    (W.D2Q9, (64, 64, 1), 0.8, (0, 0, 0), (0, 0, 0), 50, "tg"),
    (W.D2Q9, (45, 37, 1), 0.7, (0, 0, 0), (1e-5, -2e-5, 0), 21, "tg"),
]


@pytest.mark.parametrize("aa", [False, True], ids=["AB", "AA"])
@pytest.mark.parametrize("case", CASES_3D, ids=_case_id)
def test_fp64_parity_against_oracle(case, aa):
    lattice, dims, tau, bc, force, steps, kind = case
    rho, u, noise = inputs(lattice, dims, kind, seed=3, noise_amp=1e-5, bc=bc, U0=0.03)
    f_or, r_or, u_or, red_or = run_oracle(lattice, dims, tau, force, bc, rho, u, noise, steps)
    f, r, v, red = run_gpu(lattice, dims, tau, force, bc, rho, u, noise, steps, aa=aa)
    ef, eu, er = rel_err(f, f_or), rel_err(v, u_or), rel_err(r, r_or)
    print(f"{dims} bc={bc} aa={aa}: f {ef:.2e} u {eu:.2e} rho {er:.2e}")
    assert ef <= TOL and eu <= TOL and er <= TOL
    assert abs(red["mass"] - red_or["mass"]) <= TOL * abs(red_or["mass"])
    assert abs(red["ke"] - red_or["ke"]) <= 1e-10 * red_or["ke"]
    assert abs(red["umax"] - red_or["umax"]) <= TOL * red_or["umax"]
    assert not red["unstable"]


@pytest.mark.parametrize("aa", [False, True], ids=["AB", "AA"])
def test_taylor_green_2d_full_workload(aa):
    """Workload D2Q9 128^2, tau = 0.8, 1000 steps: parity at every node, and
    the kinetic energy decay rate 4 nu k^2 of the closed form."""
    n, tau, steps = 128, 0.8, 1000
    rho, u = W.taylor_green_2d(n, U0=0.01)
    f_or, r_or, u_or, red_or = run_oracle(W.D2Q9, (n, n, 1), tau, (0, 0, 0), (0, 0, 0), rho, u,
                                          None, steps)
    sim = lbm.LBM(lbm.D2Q9, n, n, 1, tau, aa=aa)
    sim.init_equilibrium(rho, u)
    ts, ke = [], []
    for it in range(steps + 1):
        if it % 10 == 0 and it >= 100:
            ts.append(it)
            ke.append(sim.reduce()["ke"])
        if it < steps:
            sim.step(1)
    f = sim.get_populations().cpu().numpy()
    _, v = sim.moments()
    assert rel_err(f, f_or) <= TOL
    assert rel_err(v.cpu().numpy(), u_or) <= TOL
    rate = -np.polyfit(np.array(ts, float), np.log(ke), 1)[0]
    nu, k = (tau - 0.5) / 3, 2 * math.pi / n
    assert abs(rate / (4 * nu * k * k) - 1) < 1e-4
    assert abs(ke[-1] - red_or["ke"]) <= 1e-10 * red_or["ke"]


@pytest.mark.parametrize("aa", [False, True], ids=["AB", "AA"])
@pytest.mark.parametrize("lattice,dims", [(W.D3Q19, (6, 6, 6)), (W.D2Q9, (9, 9, 1))])
def test_pure_streaming_bit_exact(lattice, dims, aa):
    """tau = inf: each step is the propagation permutation; the GPU equals the
    oracle bit for bit and n steps on a periodic n-cube are the identity."""
    nx, ny, nz = dims
    Q = 19 if lattice == W.D3Q19 else 9
    f0 = np.random.default_rng(1).uniform(0.0, 0.1, size=(Q, nz, ny, nx))
    sim = lbm.LBM(lattice, nx, ny, nz, math.inf, aa=aa)
    sim.set_populations(f0)
    import oracle
    ref = oracle.Sim(lattice, nx, ny, nz, tau=math.inf)
    ref.set_populations(f0)
    for k in range(1, nx + 1):
        sim.step(1)
        ref.step(1)
        assert np.array_equal(sim.get_populations().cpu().numpy(), ref.get_populations())
    assert np.array_equal(sim.get_populations().cpu().numpy(), f0)


@pytest.mark.parametrize("bc,force", [((0, 0, 0), (0, 0, 0)), ((0, 1, 0), (1e-5, 0, 0)),
                                      ((2, 1, 1), (1e-5, 1e-6, -1e-6))])
def test_aa_equals_ab_bitwise(bc, force):
    """The AA pattern runs the same collision on the same populations, so it
    matches the two-lattice scheme bit for bit after any number of steps."""
    dims = (45, 18, 13)
    rho, u, noise = inputs(W.D3Q19, dims, "channel", seed=4, noise_amp=1e-5, bc=bc, U0=0.03)
    ab = lbm.LBM(lbm.D3Q19, *dims, 0.7, force=force, bc=bc)
    aa = lbm.LBM(lbm.D3Q19, *dims, 0.7, force=force, bc=bc, aa=True)
    for s in (ab, aa):
        s.init_equilibrium(rho, u, noise)
    for n in (1, 1, 2, 3, 7):
        ab.step(n)
        aa.step(n)
        assert torch.equal(ab.get_populations(), aa.get_populations())
        assert torch.equal(ab.moments()[1], aa.moments()[1])


@pytest.mark.parametrize("lattice,dims", [
    (W.D3Q19, (2, 1024, 512)), (W.D3Q19, (34, 200, 155)), (W.D3Q19, (128, 96, 86)),
    (W.D3Q19, (1030, 33, 31)), (W.D2Q9, (18, 58255, 1)), (W.D2Q9, (514, 2048, 1)),
], ids=lambda v: str(v))
@pytest.mark.parametrize("force,comp", [((0, 0, 0), False), ((1e-5, -2e-5, 0), False),
                                        ((1e-5, 0, 0), True)], ids=["plain", "force", "comp"])
def test_two_node_kernels_ab_equals_aa_bitwise_and_oracle(lattice, dims, force, comp):
    """Periodic FP64 D2Q9 and D3Q19 steps of an even-nx box of at least 2^20
    nodes run two nodes per work-item (16-byte accesses, x-shift across lanes; rows inside
    a wavefront, rows over several workgroups, idle work-items), in the
    two-lattice pattern and in the in-place AA pattern, whose odd step also
    writes across lanes.  The two patterns apply the same collision to the
    same populations, so the states agree bit for bit after every step
    count (both AA parities), and both match the oracle.  An all-fluid solid
    mask sends the same box through the one-node kernels (masks are read
    per node), which must agree bit for bit too."""
    assert dims[0] % 2 == 0 and dims[0] * dims[1] * dims[2] >= 1 << 20
    rho, u, noise = inputs(lattice, dims, "channel", seed=12, noise_amp=1e-5, bc=(0, 0, 0), U0=0.03)
    ab = lbm.LBM(lattice, *dims, 0.7, force=force, compressible=comp)
    aa = lbm.LBM(lattice, *dims, 0.7, force=force, compressible=comp, aa=True)
    one = lbm.LBM(lattice, *dims, 0.7, force=force, compressible=comp)
    one.set_solid(np.zeros(dims[::-1], dtype=np.uint8))
    for s in (ab, aa, one):
        s.init_equilibrium(rho, u, noise)
    for n in (1, 2, 4):
        ab.step(n)
        aa.step(n)
        one.step(n)
        f_ab = ab.get_populations()
        assert torch.equal(f_ab, aa.get_populations())
        assert torch.equal(f_ab, one.get_populations())
    one.close()
    f_or, _, u_or, _ = run_oracle(lattice, dims, 0.7, force, (0, 0, 0), rho, u, noise, 7,
                                  compressible=comp)
    assert rel_err(ab.get_populations().cpu().numpy(), f_or) <= TOL
    assert rel_err(ab.moments()[1].cpu().numpy(), u_or) <= TOL


def _narrow_storage_kernels_agree(storage, lattice, dims, force, comp, counts):
    """The two-lattice step of a periodic box in `storage` (f - w), the AA
    pattern and an all-fluid solid mask (per-node kernels) from one state
    exactly representable in the storage: bit for bit after every count of
    one-step launches, and the first step within one storage ulp + FP32
    arithmetic of the FP64 oracle's step."""
    import oracle
    rho, u, noise = inputs(lattice, dims, "channel", seed=31, noise_amp=1e-4, bc=(0, 0, 0), U0=0.04)
    ref = oracle.Sim(lattice, *dims, tau=0.7, force=force, compressible=comp)
    ref.init_equilibrium(rho, u, noise)
    del rho, u, noise
    _, t = oracle.lattice_tables(lattice)
    tw = t[:, None, None, None] * np.ones((1,) + tuple(dims[::-1]))
    g0 = quantize(ref.get_populations() - tw, storage)
    g0[np.abs(g0) < 1e-8] = 0.0
    f0 = g0 + tw
    del g0
    ref.set_populations(f0)
    sims = [lbm.LBM(lattice, *dims, 0.7, force=force, storage=storage, compressible=comp, aa=aa)
            for aa in (False, True, False)]
    sims[2].set_solid(np.zeros(dims[::-1], dtype=np.uint8))
    for s in sims:
        s.set_populations(f0)
    del f0
    ref.step(1)
    g_ref = ref.get_populations() - tw
    ref.close()
    for k, n in enumerate(counts):
        for s in sims:
            for _ in range(n):  # one step per launch (D2Q9 would fuse lbm_step(n >= 4))
                s.step(1)
        f = sims[0].get_populations()
        assert torch.equal(f, sims[1].get_populations())
        assert torch.equal(f, sims[2].get_populations())
        if k == 0:
            g = f.cpu().numpy() - tw
            tol = ulp(g_ref, storage) + 64 * np.finfo(np.float32).eps * np.abs(g_ref).max()
            worst = (np.abs(g - g_ref) / tol).max()
            print(f"  first step: worst error / tolerance = {worst:.3f}", flush=True)
            assert worst <= 1.0
        del f
    for s in sims:
        s.close()


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16", "e4m11"])
@pytest.mark.parametrize("lattice,dims", [
    (W.D3Q19, (2, 1024, 512)), (W.D3Q19, (34, 200, 155)), (W.D3Q19, (128, 96, 86)),
    (W.D3Q19, (1030, 33, 31)), (W.D2Q9, (18, 58255, 1)), (W.D2Q9, (514, 2048, 1)),
    (W.D3Q19, (512, 64, 32)),
], ids=lambda v: str(v))
@pytest.mark.parametrize("force,comp", [((0, 0, 0), False), ((1e-5, -2e-5, 0), False),
                                        ((1e-5, 0, 0), True)], ids=["plain", "force", "comp"])
def test_large_narrow_storage_steps_equal_per_node_steps_and_oracle(storage, lattice, dims, force,
                                                                    comp):
    """Periodic boxes of 2^20 nodes and more in FP32, FP16, BF16 or e4m11
    storage, in the shapes of the two-node FP64 test: their two-lattice
    steps (one node per work-item, with row addressing at nx = 128 for FP32
    and e4m11) against the AA pattern and an all-fluid mask, and the
    oracle."""
    assert dims[0] * dims[1] * dims[2] >= 1 << 20
    print(f"large narrow {lattice} {dims} {storage} F={force} comp={comp}", flush=True)
    _narrow_storage_kernels_agree(storage, lattice, dims, force, comp, (1, 1, 2))


@pytest.mark.parametrize("storage", ["f32", "e4m11"])
@pytest.mark.parametrize("lattice,dims", [
    (W.D2Q9, (64, 50, 1)), (W.D3Q19, (64, 24, 10)), (W.D3Q19, (256, 5, 3)), (W.D3Q27, (128, 9, 7)),
    (W.D3Q19, (512, 8, 3)), (W.D2Q9, (1024, 16, 1)),
], ids=lambda v: str(v))
@pytest.mark.parametrize("force,comp", [((0, 0, 0), False), ((1e-5, -2e-5, 0), False),
                                        ((1e-5, 0, 0), True)], ids=["plain", "force", "comp"])
def test_row_addressed_steps_equal_per_node_steps_and_oracle(storage, lattice, dims, force, comp):
    """Periodic boxes with nx a power of two (64 to the tile length) in FP32
    or e4m11 storage step one node per work-item with the addresses of the
    source rows computed once per wavefront (rows of one and of several
    wavefronts, rows of two and four workgroups on one XCD each; D2Q9,
    D3Q19, D3Q27).  The AA pattern and an all-fluid solid mask take the
    per-node kernels, which apply the same collision to the same
    populations: all three agree bit for bit after 1, 2, 3 and 6 steps.
    From a state exactly representable in the storage format, the first step
    is the FP64 oracle's step rounded to the format, within one unit in the
    last place plus FP32 arithmetic error."""
    import oracle
    print(f"row-addressed {lattice} {dims} {storage} F={force} comp={comp}", flush=True)
    rho, u, noise = inputs(lattice, dims, "channel", seed=31, noise_amp=1e-4, bc=(0, 0, 0), U0=0.04)
    ref = oracle.Sim(lattice, *dims, tau=0.7, force=force, compressible=comp)
    ref.init_equilibrium(rho, u, noise)
    _, t = oracle.lattice_tables(lattice)
    tw = t[:, None, None, None] * np.ones((1,) + rho.shape)
    g0 = quantize(ref.get_populations() - tw, storage)
    g0[np.abs(g0) < 1e-8] = 0.0
    f0 = g0 + tw
    ref.set_populations(f0)
    sims = [lbm.LBM(lattice, *dims, 0.7, force=force, storage=storage, compressible=comp, aa=aa)
            for aa in (False, True, False)]
    sims[2].set_solid(np.zeros(dims[::-1], dtype=np.uint8))
    for s in sims:
        s.set_populations(f0)
    ref.step(1)
    g_ref = ref.get_populations() - tw
    ref.close()
    for k, n in enumerate((1, 1, 1, 3)):
        for s in sims:
            for _ in range(n):  # one step per launch (D2Q9 would fuse lbm_step(n >= 4))
                s.step(1)
        f = sims[0].get_populations()
        assert torch.equal(f, sims[1].get_populations())
        assert torch.equal(f, sims[2].get_populations())
        if k == 0:
            g = f.cpu().numpy() - tw
            tol = ulp(g_ref, storage) + 64 * np.finfo(np.float32).eps * np.abs(g_ref).max()
            worst = (np.abs(g - g_ref) / tol).max()
            print(f"  first step: worst error / tolerance = {worst:.3f}", flush=True)
            assert worst <= 1.0
    for s in sims:
        s.close()


@pytest.mark.parametrize("storage", ["f64", "f32", "f16", "bf16", "e4m11"])
@pytest.mark.parametrize("dims", [(128, 128, 1), (130, 97, 1), (7, 5, 1), (1, 1, 1), (3, 40, 1),
                                  (200, 170, 1), (3000, 200, 1), (514, 2048, 1)],
                         ids=lambda d: f"{d[0]}x{d[1]}")
@pytest.mark.parametrize("force,comp", [((0, 0, 0), False), ((1e-5, -2e-5, 0), False),
                                        ((1e-5, 0, 0), True)], ids=["plain", "force", "comp"])
def test_fused_d2q9_launches_equal_one_step_launches(storage, dims, force, comp):
    """A periodic D2Q9 two-lattice lbm_step(n) runs launches of four steps
    (16 x 16 regions in LDS, inner 8 x 8 nodes stored) in pairs and the
    remainder one step per launch; lbm_step(1) always launches one step.
    The states agree bit for bit after 8, 13 and 16 steps: on ragged boxes,
    boxes smaller than a region (wrapped several times), 16 x 16 regions in
    XCD-aware tiles of 8 x 8 blocks (partial tiles, padding workgroups; 200 x
    170), 32 x 32 regions of four nodes per work-item on large ragged boxes
    (3000 x 200, and 514 x 2048, a box of 2^20 nodes whose one-step launches
    use the two-node kernel), and every storage, where each fused step
    rounds through the storage type."""
    print(f"fused D2Q9 {dims} {storage} F={force} comp={comp}", flush=True)
    rho, u, noise = inputs(W.D2Q9, dims, "channel", seed=21, noise_amp=1e-5, bc=(0, 0, 0), U0=0.03)
    fused = lbm.LBM(lbm.D2Q9, *dims, 0.7, force=force, storage=storage, compressible=comp)
    single = lbm.LBM(lbm.D2Q9, *dims, 0.7, force=force, storage=storage, compressible=comp)
    for s in (fused, single):
        s.init_equilibrium(rho, u, noise)
    for n in (8, 13, 16):
        fused.step(n)
        for _ in range(n):
            single.step(1)
        assert fused.steps_taken == single.steps_taken
        assert torch.equal(fused.get_populations(), single.get_populations())
    fused.close()
    single.close()


@pytest.mark.parametrize("storage", ["f64", "f16", "e4m11"])
@pytest.mark.parametrize("dims", [(1000, 1100, 1), (4097, 257, 1), (256, 4096, 1), (1030, 1024, 1)],
                         ids=lambda d: f"{d[0]}x{d[1]}")
@pytest.mark.parametrize("force,comp", [((0, 0, 0), False), ((1e-5, -2e-5, 0), False),
                                        ((1e-5, 0, 0), True)], ids=["plain", "force", "comp"])
def test_streamed_d2q9_launches_equal_one_step_launches(storage, dims, force, comp):
    """Periodic D2Q9 boxes of at least 2^20 nodes run their four-step
    launches as strips of 224 stored columns streamed up row segments
    (stream2d.hpp): ragged strips and segments, a strip wider than the part
    of the box it stores (nx = 256: the second strip wraps), and segment
    lengths the launch plan picks for each box.  The state after
    8, 12 and 16 steps equals that of one-step launches bit for bit."""
    print(f"streamed D2Q9 {dims} {storage} F={force} comp={comp}", flush=True)
    rho, u, noise = inputs(W.D2Q9, dims, "channel", seed=23, noise_amp=1e-5, bc=(0, 0, 0), U0=0.03)
    fused = lbm.LBM(lbm.D2Q9, *dims, 0.7, force=force, storage=storage, compressible=comp)
    single = lbm.LBM(lbm.D2Q9, *dims, 0.7, force=force, storage=storage, compressible=comp)
    for s in (fused, single):
        s.init_equilibrium(rho, u, noise)
    for n in (8, 12, 16):
        fused.step(n)
        for _ in range(n):
            single.step(1)
        assert torch.equal(fused.get_populations(), single.get_populations())
    fused.close()
    single.close()


def test_translation_equivariance_bitwise():
    dims = (40, 24, 20)
    nx, ny, nz = dims
    rho, u, noise = inputs(W.D3Q19, dims, "tg", noise_amp=1e-5)
    a = lbm.LBM(lbm.D3Q19, *dims, 0.6, force=(1e-6, 0, 2e-6))
    a.init_equilibrium(rho, u, noise)
    f0 = a.get_populations()
    b = lbm.LBM(lbm.D3Q19, *dims, 0.6, force=(1e-6, 0, 2e-6))
    shift = (3, 5, 7)
    b.set_populations(torch.roll(f0, shift, dims=(1, 2, 3)))
    a.step(6)
    b.step(6)
    assert torch.equal(b.get_populations(), torch.roll(a.get_populations(), shift, dims=(1, 2, 3)))


@pytest.mark.parametrize("aa", [False, True], ids=["AB", "AA"])
@pytest.mark.parametrize("bc", [(0, 0, 0), (0, 1, 0), (2, 2, 1)])
def test_state_roundtrip_bitwise(aa, bc):
    """get/set are inverse permutations of the stored state: a state exported
    after any number of steps (either AA parity) and imported into a fresh
    context continues bit for bit."""
    dims = (23, 14, 9)
    rho, u, noise = inputs(W.D3Q19, dims, "channel", seed=8, noise_amp=1e-5, bc=bc, U0=0.03)
    a = lbm.LBM(lbm.D3Q19, *dims, 0.8, force=(1e-5, 0, 0), bc=bc, aa=aa)
    a.init_equilibrium(rho, u, noise)
    f0 = a.get_populations()
    a.set_populations(f0)
    assert torch.equal(a.get_populations(), f0)
    for n in (1, 2, 3):
        a.step(n)
        fa = a.get_populations()
        b = lbm.LBM(lbm.D3Q19, *dims, 0.8, force=(1e-5, 0, 0), bc=bc, aa=aa)
        b.set_populations(fa)
        assert torch.equal(b.get_populations(), fa)
        a.step(3)
        b.step(3)
        assert torch.equal(a.get_populations(), b.get_populations())
        b.close()


def test_full_size_taylor_green_256_sampled():
    """Workload D3Q19 256^3 FP64 (the benchmark's launch configuration), 6
    steps: sampled nodes -- including the periodic seams -- against the oracle
    run on each node's dependency window."""
    n, steps, tau = 256, 6, 0.6
    dims = (n, n, n)
    rho, u = W.taylor_green_3d(n, U0=0.05)
    noise = W.population_noise(W.D3Q19, dims, 1e-6, seed=2)
    sim = lbm.LBM(lbm.D3Q19, n, n, n, tau)
    sim.init_equilibrium(rho, u, noise)
    sim.step(steps)
    f = sim.get_populations()
    _, v = sim.moments()
    rng = np.random.default_rng(0)
    centers = [(0, 0, 0), (255, 255, 255), (0, 128, 255), (255, 0, 17), (64, 192, 3)]
    centers += [tuple(int(c) for c in rng.integers(0, n, 3)) for _ in range(5)]
    ef, eu = sampled_window_check(f, v, W.D3Q19, dims, tau, (0, 0, 0), (0, 0, 0), rho, u, noise,
                                  steps, centers)
    print(f"256^3 sampled: f {ef:.2e} u {eu:.2e}")
    assert ef <= TOL and eu <= TOL
    red = sim.reduce()
    assert not red["unstable"]
    assert abs(red["mass"] / (rho.sum() + noise.sum()) - 1) < 1e-13


def test_full_size_channel_sampled():
    """Workload D3Q19 channel 512 x 128 x 128, walls at y = 0 and 127, g_x =
    1e-6, tau = 0.9: sampled columns against the oracle on their dependency
    window (the full wall-normal extent)."""
    dims = (512, 128, 128)
    bc = (W.PERIODIC, W.SOLID_ENDS, W.PERIODIC)
    steps, tau, force = 4, 0.9, (1e-6, 0, 0)
    rho, u = W.channel(*dims, amplitude=1e-4, seed=3, bc=bc)
    sim = lbm.LBM(lbm.D3Q19, *dims, tau, force=force, bc=bc)
    sim.init_equilibrium(rho, u)
    sim.step(steps)
    f = sim.get_populations()
    _, v = sim.moments()
    centers = [(0, 1, 0), (511, 126, 127), (255, 64, 64), (100, 2, 3), (7, 125, 90)]
    ef, eu = sampled_window_check(f, v, W.D3Q19, dims, tau, force, bc, rho, u, None, steps,
                                  centers)
    print(f"channel sampled: f {ef:.2e} u {eu:.2e}")
    assert ef <= TOL and eu <= TOL


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16", "e4m11"])
@pytest.mark.parametrize("aa", [False, True], ids=["AB", "AA"])
def test_reduced_precision_one_step(storage, aa):
    """Deviation storage: from a state exactly representable in the storage
    format, one step equals the FP64 oracle's step rounded to the format, to
    within one unit in the last place of the format plus FP32 arithmetic
    error."""
    import oracle
    dims = (37, 21, 10)
    bc, force, tau = (0, 1, 0), (1e-5, 0, 0), 0.7
    rho, u, noise = inputs(W.D3Q19, dims, "channel", seed=9, noise_amp=1e-4, bc=bc, U0=0.04)
    ref = oracle.Sim(W.D3Q19, *dims, tau=tau, force=force, bc=bc)
    ref.init_equilibrium(rho, u, noise)
    fluid = ref.geometry()
    _, t = oracle.lattice_tables(W.D3Q19)
    tw = t[:, None, None, None] * fluid
    g0 = quantize(ref.get_populations() - tw, storage)
    g0[np.abs(g0) < 1e-8] = 0.0
    f0 = g0 + tw
    ref.set_populations(f0)
    sim = lbm.LBM(lbm.D3Q19, *dims, tau, force=force, bc=bc, storage=storage, aa=aa)
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


def test_reduce_flags_non_finite():
    dims = (8, 6, 5)
    sim = lbm.LBM(lbm.D3Q19, *dims, 0.8)
    rho, u, _ = inputs(W.D3Q19, dims, "tg", noise_amp=0)
    sim.init_equilibrium(rho, u)
    f = sim.get_populations()
    f[3, 2, 1, 4] = float("nan")
    sim.set_populations(f)
    assert sim.reduce()["unstable"]
    sim.set_populations(torch.nan_to_num(f, nan=1.0 / 36))
    assert not sim.reduce()["unstable"]


def test_error_paths_on_device():
    sim = lbm.LBM(lbm.D3Q19, 8, 8, 8, 0.8)
    with pytest.raises(lbm.LBMError) as e:
        sim.step(1)  # no state yet
    assert e.value.status == lbm.ESTATE
    sim.init_equilibrium(np.ones((8, 8, 8)), np.zeros((3, 8, 8, 8)))
    sim.step(0)
    assert sim.steps_taken == 0
    with pytest.raises(lbm.LBMError) as e:
        sim.step(-1)
    assert e.value.status == lbm.EINVAL
    host = torch.zeros((19, 8, 8, 8), dtype=torch.float64)
    st = lbm.lib().lbm_get_populations(sim._h, host.data_ptr())
    assert st == lbm.EINVAL  # host pointer rejected before any launch


def test_runs_on_a_side_stream():
    dims = (20, 12, 10)
    rho, u, noise = inputs(W.D3Q19, dims, "tg", noise_amp=1e-5)
    ref = run_gpu(W.D3Q19, dims, 0.7, (0, 0, 0), (0, 0, 0), rho, u, noise, 8, reduce=False)[0]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        sim = lbm.LBM(lbm.D3Q19, *dims, 0.7)
        sim.init_equilibrium(rho, u, noise)
        sim.step(8)
        f = sim.get_populations()
    s.synchronize()
    assert np.array_equal(f.cpu().numpy(), ref)


def test_context_stream_differs_from_the_current_stream():
    """A context bound to a side stream, driven from the default stream with
    host inputs (copied on the default stream) and outputs consumed there
    without an explicit synchronisation: the binding orders the two streams,
    and the results equal a run on one stream."""
    dims = (64, 48, 40)
    rho, u, noise = inputs(W.D3Q19, dims, "tg", noise_amp=1e-5)
    ref = run_gpu(W.D3Q19, dims, 0.7, (1e-6, 0, 0), (0, 0, 0), rho, u, noise, 9, reduce=False)
    side = torch.cuda.Stream()
    sim = lbm.LBM(lbm.D3Q19, *dims, 0.7, force=(1e-6, 0, 0), stream=side)
    for _ in range(3):
        sim.init_equilibrium(rho, u, noise)
        sim.step(9)
        f = sim.get_populations()
        r, v = sim.moments()
        total = (f * 2.0).sum()  # consumed on the default stream
        assert np.array_equal(f.cpu().numpy(), ref[0])
        assert np.array_equal(v.cpu().numpy(), ref[2])
        assert torch.isfinite(total).item()
    sim.close()


@pytest.mark.parametrize("n", [128, 512])
@pytest.mark.parametrize("aa", [False, True], ids=["AB", "AA"])
def test_graph_replay_matches_eager_bitwise(aa, n):
    """LBM_FLAG_GRAPH replays a captured 32-step graph: after step counts that
    mix replays, parity alignment and eager remainders -- with eager work
    (reductions, exports) between replays -- the state equals the eager run
    bit for bit every time.  Two-lattice D2Q9 graphs hold four-step launches
    (16 x 16 regions at 128^2, 32 x 32 regions at 512^2)."""
    rho, u = W.taylor_green_2d(n, U0=0.01)
    g = lbm.LBM(lbm.D2Q9, n, n, 1, 0.8, aa=aa, graph=True)
    e = lbm.LBM(lbm.D2Q9, n, n, 1, 0.8, aa=aa)
    for s in (g, e):
        s.init_equilibrium(rho, u)
    for k in (100, 7, 64, 33, 1, 32, 200):
        g.step(k)
        e.step(k)
        assert g.steps_taken == e.steps_taken
        assert g.reduce() == e.reduce()
        assert torch.equal(g.get_populations(), e.get_populations())


@pytest.mark.parametrize("aa", [False, True], ids=["AB", "AA"])
def test_graph_replay_of_two_node_kernels(aa):
    """The captured graph of a periodic FP64 box of 2^20 nodes holds the
    two-node kernels; replays equal the eager run bit for bit."""
    dims = (128, 128, 64)
    rho, u = W.taylor_green_3d(*dims, U0=0.05)
    g = lbm.LBM(lbm.D3Q19, *dims, 0.6, aa=aa, graph=True)
    e = lbm.LBM(lbm.D3Q19, *dims, 0.6, aa=aa)
    for s in (g, e):
        s.init_equilibrium(rho, u)
    for k in (33, 64, 5):
        g.step(k)
        e.step(k)
        assert torch.equal(g.get_populations(), e.get_populations())


def test_buffers_too_small_for_the_call_are_rejected():
    """Every device buffer is checked against the allocation that holds it
    (hipMemGetAddressRange) before any launch: buffers too small for what
    the call reads or writes give LBM_EINVAL, and the context stays usable."""
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    dims = (64, 64, 32)
    N = 64 * 64 * 32
    rho = torch.ones(dims[::-1], dtype=torch.float64, device="cuda")
    u = torch.zeros((3,) + dims[::-1], dtype=torch.float64, device="cuda")
    sim = lbm.LBM(lbm.D3Q19, *dims, 0.7)
    sim.init_equilibrium(rho, u)
    L = lbm.lib()
    small = ctypes.c_void_p()
    assert hip.hipMalloc(ctypes.byref(small), ctypes.c_size_t(8 * N)) == 0  # one FP64 field
    try:
        assert L.lbm_set_populations(sim._h, small) == lbm.EINVAL  # needs Q fields
        assert b"needs" in L.lbm_last_error()
        assert L.lbm_get_populations(sim._h, small) == lbm.EINVAL
        assert L.lbm_init_equilibrium(sim._h, small, small, None) == lbm.EINVAL  # u is [3][N]
        off = ctypes.c_void_p(small.value + 8)  # one element short of a field
        assert L.lbm_moments(sim._h, off, None, 0) == lbm.EINVAL
        assert L.lbm_moments(sim._h, small, None, 0) == lbm.OK  # exactly one field
        ctx = ctypes.c_void_p()
        F = (ctypes.c_double * 3)()
        assert L.lbm_create(ctypes.byref(ctx), lbm.D3Q19, *dims, 0.7, F, None, lbm.F64, 0) == lbm.OK
        assert L.lbm_bind(ctx, small, small, None) == lbm.EINVAL  # not a population buffer
        L.lbm_destroy(ctx)
        sim.step(2)
        assert sim.reduce()["mass"] > 0
    finally:
        torch.cuda.synchronize()
        hip.hipFree(small)
