"""Seeded synthetic inputs of the workloads (initial fields and perturbations).

This module holds no arithmetic of the method itself: it only produces the
given fields that the paper's InitUP supplies (Sec. 2.2, Sec. 3.1) -- a
density rho = p/c_s^2, a velocity u, and optional perturbation arrays -- and
hands the same arrays to the GPU library and to the CPU oracle.  All arrays
are numpy float64 in the canonical order [component][z][y][x].

The paper's own workloads are analytic flows (a cylinder and a sphere in a
channel, Sec. 4-6); the fields here are analytic flows of the same kind that
need no inlet/outlet boundary scheme: Taylor-Green vortices, a forced
channel, and a random divergence-free field.
"""
import math

import numpy as np

D2Q9, D3Q19, D3Q27 = 0, 1, 2
PERIODIC, SOLID_ENDS, WALLS_OUTSIDE, WALLS_NODAL = 0, 1, 2, 3
Q_OF = {D2Q9: 9, D3Q19: 19, D3Q27: 27}


def _grid(n):
    """Node angles x_i = 2*pi*i/n, i = 0..n-1."""
    return 2.0 * math.pi * np.arange(n, dtype=np.float64) / n


def taylor_green_2d(n=128, U0=0.01):
    """2D Taylor-Green vortex on an n x n periodic grid (nz = 1):
    u = U0 sin(kx) cos(ky), v = -U0 cos(kx) sin(ky), k = 2 pi / n, and the
    matching pressure p = p0 + (U0^2/4)(cos 2kx + cos 2ky), given here as
    rho = p/c_s^2 = 1 + 3 (U0^2/4)(cos 2kx + cos 2ky)."""
    x = _grid(n)[None, None, :]
    y = _grid(n)[None, :, None]
    shape = (1, n, n)
    u = np.zeros((3,) + shape)
    u[0] = np.broadcast_to(U0 * np.sin(x) * np.cos(y), shape)
    u[1] = np.broadcast_to(-U0 * np.cos(x) * np.sin(y), shape)
    rho = np.broadcast_to(1.0 + 3.0 * (U0 * U0 / 4.0) * (np.cos(2 * x) + np.cos(2 * y)), shape)
    return np.ascontiguousarray(rho), u


def taylor_green_3d(nx, ny=None, nz=None, U0=0.05):
    """3D Taylor-Green vortex: u = U0 sin x cos y cos z, v = -U0 cos x sin y
    cos z, w = 0 on the 2 pi / n grid of each axis, with pressure
    p = p0 + (U0^2/16)(cos 2x + cos 2y)(cos 2z + 2), i.e.
    rho = 1 + 3 (U0^2/16)(cos 2x + cos 2y)(cos 2z + 2)."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    x = _grid(nx)[None, None, :]
    y = _grid(ny)[None, :, None]
    z = _grid(nz)[:, None, None]
    shape = (nz, ny, nx)
    u = np.zeros((3,) + shape)
    u[0] = U0 * np.sin(x) * np.cos(y) * np.cos(z)
    u[1] = -U0 * np.cos(x) * np.sin(y) * np.cos(z)
    rho = 1.0 + 3.0 * (U0 * U0 / 16.0) * (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0)
    return np.ascontiguousarray(np.broadcast_to(rho, shape)), u


def uniform_noise(shape, amplitude, seed):
    """Independent U(-A, +A) values (numpy PCG64, ``default_rng(seed)``)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-amplitude, amplitude, size=shape)


def uniform_noise_device(shape, amplitude, seed, device="cuda"):
    """Independent U(-A, +A) values generated on a device with torch's seeded
    generator (for fields too large to build on the host)."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(seed)
    t = torch.empty(shape, dtype=torch.float64, device=device)
    t.uniform_(-amplitude, amplitude, generator=g)
    return t


def population_noise(lattice, dims, amplitude, seed):
    """Perturbation added to every population of every node, [Q][z][y][x]."""
    nx, ny, nz = dims
    return uniform_noise((Q_OF[lattice], nz, ny, nx), amplitude, seed)


def solid_mask(dims, bc):
    """Nodes on the first and last plane of an axis with solid ends."""
    nx, ny, nz = dims
    solid = np.zeros((nz, ny, nx), dtype=bool)
    if bc[0] == SOLID_ENDS:
        solid[:, :, 0] = solid[:, :, -1] = True
    if bc[1] == SOLID_ENDS:
        solid[:, 0, :] = solid[:, -1, :] = True
    if bc[2] == SOLID_ENDS:
        solid[0, :, :] = solid[-1, :, :] = True
    return solid


def channel(nx=512, ny=128, nz=128, amplitude=1e-4, seed=3, bc=(PERIODIC, SOLID_ENDS, PERIODIC)):
    """Forced channel start: rho = 1 and a velocity of independent U(-A, +A)
    components on the fluid nodes (zero on solid nodes)."""
    rho = np.ones((nz, ny, nx))
    u = uniform_noise((3, nz, ny, nx), amplitude, seed)
    u[:, solid_mask((nx, ny, nz), bc)] = 0.0
    return rho, u


def random_fourier_field(n=128, modes=8, kmax=4, amplitude=0.02, seed=11, dims=3):
    """Divergence-free random field: sum over ``modes`` Fourier modes of
    amplitude * a_m cos(2 pi K_m . x / n + phi_m), with K_m drawn uniformly
    from the nonzero integer vectors with |K| <= kmax, a_m a random unit
    vector orthogonal to K_m, phi_m ~ U[0, 2 pi).  Each mode is divergence
    free because a_m . K_m = 0."""
    rng = np.random.default_rng(seed)
    r = np.arange(-kmax, kmax + 1)
    if dims == 3:
        cand = np.array([(a, b, c) for a in r for b in r for c in r
                         if 0 < a * a + b * b + c * c <= kmax * kmax], dtype=np.float64)
    else:
        cand = np.array([(a, b, 0) for a in r for b in r if 0 < a * a + b * b <= kmax * kmax],
                        dtype=np.float64)
    nzs = n if dims == 3 else 1
    idx = np.arange(n, dtype=np.float64)
    X = idx[None, None, :]
    Y = idx[None, :, None]
    Z = np.arange(nzs, dtype=np.float64)[:, None, None]
    u = np.zeros((3, nzs, n, n))
    for _ in range(modes):
        K = cand[rng.integers(len(cand))]
        v = rng.normal(size=3)
        if dims == 2:
            v[2] = 0.0
        v -= K * (v @ K) / (K @ K)
        a = v / np.linalg.norm(v)
        phi = rng.uniform(0.0, 2.0 * math.pi)
        phase = 2.0 * math.pi * (K[0] * X + K[1] * Y + K[2] * Z) / n + phi
        c = np.cos(phase)
        for d in range(3):
            u[d] += amplitude * a[d] * c
    rho = np.ones((nzs, n, n))
    return rho, u


def sphere_mask(dims, center, radius):
    """Solid nodes of a sphere: |x - center| <= radius (node coordinates).
    The paper's validation obstacle is r = 8 at (64, 64, 64) in a
    512 x 128 x 128 box (Sec. 5)."""
    nx, ny, nz = dims
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r2 = (x - center[0]) ** 2 + (y - center[1]) ** 2 + (z - center[2]) ** 2
    return (r2 <= radius * radius).astype(np.uint8)
