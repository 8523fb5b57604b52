"""Helpers shared by the GPU parity tests: run the HIP path and the CPU oracle
on the same seeded inputs and compare."""
import numpy as np
import torch

import oracle
from paper_2201_11330_amd import lbm
from paper_2201_11330_amd import workloads as W


def rel_err(got, ref):
    """max |got - ref| / max |ref| (the parity metric, relative to the field's scale)."""
    scale = np.abs(ref).max()
    return np.abs(got - ref).max() / (scale if scale > 0 else 1.0)


def inputs(lattice, dims, kind="tg", seed=2, noise_amp=1e-6, bc=(0, 0, 0), U0=0.05):
    nx, ny, nz = dims
    if kind == "tg":
        if lattice == W.D2Q9:
            rho, u = W.taylor_green_2d(nx, U0=U0) if nx == ny else W.taylor_green_3d(nx, ny, 1, U0=U0)
            if nx != ny:
                u[2] = 0.0
        else:
            rho, u = W.taylor_green_3d(nx, ny, nz, U0=U0)
    else:
        rho, u = W.channel(nx, ny, nz, amplitude=U0, seed=seed, bc=bc)
        if lattice == W.D2Q9:
            u[2] = 0.0
    noise = W.population_noise(lattice, dims, noise_amp, seed + 100) if noise_amp else None
    return rho, u, noise


def run_oracle(lattice, dims, tau, force, bc, rho, u, noise, steps, solid=None,
               compressible=False):
    s = oracle.Sim(lattice, *dims, tau=tau, force=force, bc=bc, compressible=compressible)
    if solid is not None:
        s.set_solid(solid)
    s.init_equilibrium(rho, u, noise)
    s.step(steps)
    f = s.get_populations()
    r, v = s.moments()
    red = s.reduce()
    s.close()
    return f, r, v, red


def run_gpu(lattice, dims, tau, force, bc, rho, u, noise, steps, storage="f64", aa=False,
            reduce=True, solid=None, compressible=False):
    sim = lbm.LBM(lattice, *dims, tau, force=force, bc=bc, storage=storage, aa=aa,
                  compressible=compressible)
    if solid is not None:
        sim.set_solid(solid)
    sim.init_equilibrium(rho, u, noise)
    sim.step(steps)
    f = sim.get_populations().cpu().numpy()
    r, v = sim.moments()
    red = sim.reduce() if reduce else None
    out = (f, r.cpu().numpy(), v.cpu().numpy(), red)
    sim.close()
    return out


def window_indices(center, half, n, periodic):
    """Indices of a window of half-width ``half`` around ``center`` on an axis
    of n nodes (wrapped), or the whole axis when it is not periodic."""
    if not periodic or 2 * half + 1 >= n:
        return np.arange(n), center
    return (center + np.arange(-half, half + 1)) % n, half


def sampled_window_check(f_gpu_dev, u_gpu_dev, lattice, dims, tau, force, bc, rho, u, noise,
                         steps, centers, solid=None):
    """Compares GPU outputs after ``steps`` steps at sample nodes with an oracle
    run on the dependency window of each node (half-width = steps on periodic
    axes, the full extent on wall axes).  Returns the worst errors of f and u
    relative to the field scales max |f| (the windows' largest population) and
    max |u| of the initial velocity field (plus |F|), as in the full-field
    parity metric."""
    nx, ny, nz = dims
    worst_f = worst_u = 0.0
    u_scale = max(np.abs(u).max(), np.abs(np.asarray(force, dtype=float)).max(), 1e-300)
    f_scale = 0.0
    for (cx, cy, cz) in centers:
        ix, ox = window_indices(cx, steps, nx, bc[0] == W.PERIODIC)
        iy, oy = window_indices(cy, steps, ny, bc[1] == W.PERIODIC)
        iz, oz = window_indices(cz, steps, nz, bc[2] == W.PERIODIC)
        sub = np.ix_(iz, iy, ix)
        r_w = rho[sub]
        u_w = u[(slice(None),) + sub]
        n_w = noise[(slice(None),) + sub] if noise is not None else None
        wdims = (len(ix), len(iy), len(iz))
        wbc = tuple(W.PERIODIC if (b == W.PERIODIC) else b for b in bc)
        s_w = None if solid is None else np.ascontiguousarray(solid[sub])
        f_or, _, u_or, _ = run_oracle(lattice, wdims, tau, force, wbc, np.ascontiguousarray(r_w),
                                      np.ascontiguousarray(u_w),
                                      None if n_w is None else np.ascontiguousarray(n_w), steps,
                                      solid=s_w)
        f_ref = f_or[:, oz, oy, ox]
        u_ref = u_or[:, oz, oy, ox]
        f_got = f_gpu_dev[:, cz, cy, cx].cpu().numpy()
        u_got = u_gpu_dev[:, cz, cy, cx].cpu().numpy()
        f_scale = max(f_scale, np.abs(f_or).max())
        worst_f = max(worst_f, np.abs(f_got - f_ref).max())
        worst_u = max(worst_u, np.abs(u_got - u_ref).max())
    return worst_f / f_scale, worst_u / u_scale


def round_to_bf16(x):
    """Nearest-even rounding of FP64 values to bfloat16 precision (8
    significant bits, FP32 exponent range), computed with frexp/ldexp."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)
    return np.ldexp(np.rint(np.ldexp(m, 8)), e - 8)


E4M11_MAX = 2.0 ** -1 * (2.0 - 2.0 ** -11)  # largest finite value of the 16-bit e4m11 format


def round_to_e4m11(x):
    """Nearest-even rounding of FP64 values to the e4m11 storage format: 12
    significant bits from 2^-14 up, a fixed spacing of 2^-25 below, values
    past the largest finite (2^-1 (2 - 2^-11)) to infinity; computed with
    frexp/ldexp."""
    x = np.asarray(x, dtype=np.float64)
    a = np.abs(x)
    m, e = np.frexp(a)
    normal = np.ldexp(np.rint(np.ldexp(m, 12)), e - 12)
    sub = np.ldexp(np.rint(np.ldexp(a, 25)), -25)
    q = np.where(a >= 2.0 ** -14, normal, sub)
    q = np.where(q > E4M11_MAX, np.inf, q)
    return np.copysign(q, x)


def quantize(x, storage):
    if storage == "e4m11":
        return round_to_e4m11(x)
    if storage == "f16":
        return x.astype(np.float16).astype(np.float64)
    if storage == "bf16":
        return round_to_bf16(x)
    if storage == "f32":
        return x.astype(np.float32).astype(np.float64)
    return x


def ulp(x, storage):
    """Spacing of the storage format at |x| (half-ulp is the rounding bound)."""
    a = np.abs(np.asarray(x, dtype=np.float64))
    if storage == "f16":
        return np.spacing(a.astype(np.float16)).astype(np.float64)
    if storage == "f32":
        return np.spacing(a.astype(np.float32)).astype(np.float64)
    if storage == "bf16":
        m, e = np.frexp(np.maximum(a, 1e-38))
        return np.ldexp(1.0, e - 8)
    if storage == "e4m11":
        m, e = np.frexp(np.maximum(a, 2.0 ** -14))
        return np.ldexp(1.0, e - 12)
    return np.spacing(a)


def sync():
    torch.cuda.synchronize()
