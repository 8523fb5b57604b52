"""lbm_reduce_noalloc (the Monitor reduction for callers that cannot
allocate): through the C ABI its device result equals lbm_reduce's host
outputs bit for bit, on two calls in a row with the second on a smaller box
(the static scratch keeps the first call's partials), and it writes nothing
outside its 4 doubles."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2201_11330_amd import lbm
from paper_2201_11330_amd import workloads as W

pytestmark = pytest.mark.gpu


def _sim(lattice, dims, storage, bc, force, seed):
    nx, ny, nz = dims
    sim = lbm.LBM(lattice, nx, ny, nz, 0.7, force=force, bc=bc, storage=storage)
    rho, u = W.channel(nx, ny, nz, amplitude=1e-2, seed=seed, bc=bc)
    noise = W.population_noise(lattice, dims, 1e-4, seed=seed + 1)
    sim.init_equilibrium(rho, u, noise)
    sim.step(5)
    return sim


def _noalloc(sim, guard):
    """Calls lbm_reduce_noalloc into guard[1:5]; returns the 4 results."""
    torch.cuda.synchronize()
    res = guard[1:5]
    st = lbm.lib().lbm_reduce_noalloc(sim._h, ctypes.c_void_p(res.data_ptr()))
    assert st == lbm.OK, lbm.lib().lbm_last_error()
    torch.cuda.synchronize()
    return guard.cpu().numpy()


CASES = [
    # (lattice, dims, storage, bc, force): the second of each pair is smaller
    [(lbm.D3Q19, (37, 29, 23), "f64", (W.PERIODIC, W.SOLID_ENDS, W.PERIODIC), (1e-5, 0.0, 0.0)),
     (lbm.D3Q19, (9, 7, 5), "f64", (W.PERIODIC, W.PERIODIC, W.PERIODIC), (0.0, 0.0, 0.0))],
    [(lbm.D3Q19, (64, 64, 64), "f16", (W.PERIODIC, W.PERIODIC, W.PERIODIC), (0.0, 0.0, 0.0)),
     (lbm.D2Q9, (33, 17, 1), "bf16", (W.PERIODIC, W.SOLID_ENDS, W.PERIODIC), (2e-5, 0.0, 0.0))],
]


@pytest.mark.parametrize("pair", CASES, ids=["f64-walls-then-small", "f16-then-small-d2q9-bf16"])
def test_noalloc_reduce_equals_reduce_on_two_calls(pair):
    sentinel = -12345.0
    for k, (lattice, dims, storage, bc, force) in enumerate(pair):
        sim = _sim(lattice, dims, storage, bc, force, seed=20 + 2 * k)
        guard = torch.full((6,), sentinel, dtype=torch.float64, device="cuda")
        got = _noalloc(sim, guard)
        ref = sim.reduce()
        print(f"call {k + 1} {dims} {storage}: noalloc mass {got[1]!r} ke {got[2]!r} "
              f"umax {got[3]!r}; lbm_reduce mass {ref['mass']!r} ke {ref['ke']!r} "
              f"umax {ref['umax']!r}")
        assert got[0] == sentinel and got[5] == sentinel  # nothing outside the 4 results
        assert got[1] == ref["mass"] and got[2] == ref["ke"] and got[3] == ref["umax"]
        assert got[4] == 0.0 and not ref["unstable"]
        # a second call on the same context after more steps (ordered on the stream)
        sim.step(3)
        got2 = _noalloc(sim, guard)
        ref2 = sim.reduce()
        assert got2[1] == ref2["mass"] and got2[2] == ref2["ke"] and got2[3] == ref2["umax"]
        assert got2[2] != got[2]  # the state moved on
        sim.close()


def test_noalloc_reduce_rejects_bad_result_pointers():
    sim = _sim(lbm.D3Q19, (8, 6, 4), "f64", (0, 0, 0), (0.0, 0.0, 0.0), seed=30)
    L = lbm.lib()
    assert L.lbm_reduce_noalloc(sim._h, None) == lbm.EINVAL
    host = (ctypes.c_double * 4)()
    assert L.lbm_reduce_noalloc(sim._h, ctypes.cast(host, ctypes.c_void_p)) == lbm.EINVAL
    assert b"not" in L.lbm_last_error()  # "... is not a HIP allocation" / "not device memory"
    sim.close()
