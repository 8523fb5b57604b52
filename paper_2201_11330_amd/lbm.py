"""ctypes binding of liblbm.so (include/lbm.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of the library.  PyTorch supplies device memory (tensors) and the stream.
If the library is missing the import of a binding call raises; there is no
other code path.
"""
import ctypes
import math
import os

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblbm.so")

# Enumerations of lbm.h.
D2Q9, D3Q19, D3Q27 = 0, 1, 2
PERIODIC, SOLID_ENDS, WALLS_OUTSIDE, WALLS_NODAL = 0, 1, 2, 3
F64, F32, F16_DEV, BF16_DEV, E4M11_DEV = 0, 1, 2, 3, 4
FLAG_AA, FLAG_GRAPH, FLAG_COMPRESSIBLE = 1, 2, 4
OK, EINVAL, ENOTBOUND, EHIP, EUNSTABLE, ESTATE = 0, -1, -2, -3, -4, -5

STORAGE_NAMES = {"f64": F64, "f32": F32, "f16": F16_DEV, "bf16": BF16_DEV, "e4m11": E4M11_DEV}
Q_OF = {D2Q9: 9, D3Q19: 19, D3Q27: 27}

# Every symbol include/lbm.h declares.
EXPORTS = (
    "lbm_create", "lbm_buffer_bytes", "lbm_bind", "lbm_init_equilibrium",
    "lbm_set_populations", "lbm_get_populations", "lbm_step", "lbm_moments", "lbm_reduce",
    "lbm_reduce_noalloc", "lbm_steps_taken", "lbm_set_solid", "lbm_wall_force", "lbm_forward_record",
    "lbm_adjoint_workspace_bytes", "lbm_adjoint", "lbm_destroy", "lbm_status_string",
    "lbm_last_error",
)


class LBMError(RuntimeError):
    def __init__(self, status, where, detail):
        super().__init__(f"{where}: {detail} (status {status})")
        self.status = status


class _BC(ctypes.Structure):
    _fields_ = [("axis", ctypes.c_int * 3)]


_lib = None


def lib():
    """The loaded liblbm.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                           "(python -m paper_2201_11330_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    vp, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
    st = ctypes.c_int
    L.lbm_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                             ctypes.c_int, ctypes.c_double, dp, ctypes.POINTER(_BC), ctypes.c_int,
                             ctypes.c_uint]
    L.lbm_create.restype = st
    L.lbm_buffer_bytes.argtypes = [vp]
    L.lbm_buffer_bytes.restype = ctypes.c_size_t
    L.lbm_bind.argtypes = [vp, vp, vp, vp]
    L.lbm_bind.restype = st
    L.lbm_init_equilibrium.argtypes = [vp, vp, vp, vp]
    L.lbm_init_equilibrium.restype = st
    L.lbm_set_populations.argtypes = [vp, vp]
    L.lbm_set_populations.restype = st
    L.lbm_get_populations.argtypes = [vp, vp]
    L.lbm_get_populations.restype = st
    L.lbm_step.argtypes = [vp, ctypes.c_int]
    L.lbm_step.restype = st
    L.lbm_moments.argtypes = [vp, vp, vp, ctypes.c_int]
    L.lbm_moments.restype = st
    L.lbm_reduce.argtypes = [vp, dp, dp, dp]
    L.lbm_reduce.restype = st
    L.lbm_reduce_noalloc.argtypes = [vp, vp]
    L.lbm_reduce_noalloc.restype = st
    L.lbm_steps_taken.argtypes = [vp]
    L.lbm_steps_taken.restype = ctypes.c_longlong
    L.lbm_set_solid.argtypes = [vp, vp]
    L.lbm_set_solid.restype = st
    L.lbm_wall_force.argtypes = [vp, dp]
    L.lbm_wall_force.restype = st
    L.lbm_forward_record.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp]
    L.lbm_forward_record.restype = st
    L.lbm_adjoint_workspace_bytes.argtypes = [vp, ctypes.c_int]
    L.lbm_adjoint_workspace_bytes.restype = ctypes.c_size_t
    L.lbm_adjoint.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, vp, vp, vp, vp, vp, dp, dp]
    L.lbm_adjoint.restype = st
    L.lbm_destroy.argtypes = [vp]
    L.lbm_destroy.restype = st
    L.lbm_status_string.argtypes = [ctypes.c_int]
    L.lbm_status_string.restype = ctypes.c_char_p
    L.lbm_last_error.argtypes = []
    L.lbm_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def check(status, where):
    if status != OK:
        detail = lib().lbm_last_error().decode(errors="replace")
        raise LBMError(status, where, detail or lib().lbm_status_string(status).decode())
    return status


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _dev_f64(t, shape, device):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        t = torch.from_numpy(np.require(t, dtype=np.float64, requirements=["C", "W"]))
    t = t.to(device=device, dtype=torch.float64)
    return t.reshape(shape).contiguous()


class LBM:
    """One lattice Boltzmann state on one GPU.

    ``tau`` is the lattice relaxation time (omega = 1/tau, nu = (tau - 1/2)/3);
    ``bc`` gives PERIODIC / SOLID_ENDS / WALLS_OUTSIDE / WALLS_NODAL per axis
    (x, y, z); ``storage`` is "f64", "f32", "f16", "bf16" or "e4m11"; ``aa`` selects
    the in-place AA pattern; ``graph`` makes step() replay a captured HIP
    graph of 32 steps; ``compressible`` selects the equilibrium of Eq. (feq).
    Launches go to ``stream`` (default: torch's current stream at
    construction time).
    """

    def __init__(self, lattice, nx, ny, nz, tau, force=(0.0, 0.0, 0.0), bc=(0, 0, 0),
                 storage="f64", aa=False, device=None, stream=None, graph=False,
                 compressible=False):
        L = lib()
        self.lattice = lattice
        self.Q = Q_OF[lattice]
        self.dims = (nx, ny, nz)
        self.shape = (nz, ny, nx)
        self.N = nx * ny * nz
        self.tau = float(tau)
        self.force = tuple(float(v) for v in force)
        self.bc = tuple(int(b) for b in bc)
        self.storage = STORAGE_NAMES[storage] if isinstance(storage, str) else int(storage)
        self.aa = bool(aa)
        self.compressible = bool(compressible)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        h = ctypes.c_void_p()
        F = (ctypes.c_double * 3)(*self.force)
        bcs = _BC((ctypes.c_int * 3)(*self.bc))
        check(L.lbm_create(ctypes.byref(h), lattice, nx, ny, nz, self.tau, F, ctypes.byref(bcs),
                           self.storage, (FLAG_AA if self.aa else 0) | (FLAG_GRAPH if graph else 0)
                           | (FLAG_COMPRESSIBLE if self.compressible else 0)),
              "lbm_create")
        self._h = h
        nbytes = L.lbm_buffer_bytes(h)
        self.buffers = [torch.empty(nbytes, dtype=torch.uint8, device=self.device)
                        for _ in range(1 if self.aa else 2)]
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        check(L.lbm_bind(h, _ptr(self.buffers[0]), _ptr(self.buffers[1]) if not self.aa else None,
                         ctypes.c_void_p(self.stream.cuda_stream)), "lbm_bind")
        for b in self.buffers:  # used on the context's stream until freed
            b.record_stream(self.stream)

    # -- life cycle ---------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            lib().lbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- streams ------------------------------------------------------------
    # Tensors are made (and host data copied in) on torch's current stream,
    # while the library runs on the context's stream.  Before a call the
    # context's stream waits for the current one, and every device tensor the
    # call uses is recorded on the context's stream (the caching allocator then
    # keeps its memory until that stream has passed it); after the call the
    # current stream waits for the context's stream, so results are ready
    # there.  With the default stream choice both are the same stream and
    # nothing waits.
    def _enter(self, *tensors):
        cur = torch.cuda.current_stream(self.device)
        if cur != self.stream:
            self.stream.wait_stream(cur)
        for t in tensors:
            if t is not None:
                t.record_stream(self.stream)

    def _leave(self):
        cur = torch.cuda.current_stream(self.device)
        if cur != self.stream:
            cur.wait_stream(self.stream)

    # -- state --------------------------------------------------------------
    def init_equilibrium(self, rho, u, noise=None):
        rho = _dev_f64(rho, self.shape, self.device)
        u = _dev_f64(u, (3,) + self.shape, self.device)
        noise = _dev_f64(noise, (self.Q,) + self.shape, self.device)
        self._enter(rho, u, noise)
        check(lib().lbm_init_equilibrium(self._h, _ptr(rho), _ptr(u), _ptr(noise)),
              "lbm_init_equilibrium")
        self._leave()

    def set_populations(self, f):
        f = _dev_f64(f, (self.Q,) + self.shape, self.device)
        self._enter(f)
        check(lib().lbm_set_populations(self._h, _ptr(f)), "lbm_set_populations")
        self._leave()

    def get_populations(self):
        f = torch.empty((self.Q,) + self.shape, dtype=torch.float64, device=self.device)
        self._enter(f)
        check(lib().lbm_get_populations(self._h, _ptr(f)), "lbm_get_populations")
        self._leave()
        return f

    def step(self, n=1):
        self._enter()
        check(lib().lbm_step(self._h, int(n)), "lbm_step")
        self._leave()

    @property
    def steps_taken(self):
        return lib().lbm_steps_taken(self._h)

    def moments(self, dtype=torch.float64, rho=None, u=None):
        """(rho, u) of the current state: rho = sum f, u = sum e f + F/2
        (over rho in the compressible model)."""
        if rho is None:
            rho = torch.empty(self.shape, dtype=dtype, device=self.device)
        if u is None:
            u = torch.empty((3,) + self.shape, dtype=dtype, device=self.device)
        self._enter(rho, u)
        check(lib().lbm_moments(self._h, _ptr(rho), _ptr(u), 1 if dtype == torch.float32 else 0),
              "lbm_moments")
        self._leave()
        return rho, u

    # -- geometry -------------------------------------------------------------
    def set_solid(self, solid):
        """Solid mask [nz, ny, nx] (nonzero = solid); before initialisation."""
        if not isinstance(solid, torch.Tensor):
            solid = torch.from_numpy(np.ascontiguousarray(np.asarray(solid), dtype=np.uint8))
        m = solid.to(device=self.device, dtype=torch.uint8).reshape(self.shape).contiguous()
        self._enter(m)
        check(lib().lbm_set_solid(self._h, _ptr(m)), "lbm_set_solid")
        self._leave()

    def wall_force(self):
        """Momentum-exchange force on the walls during the last propagation."""
        F = (ctypes.c_double * 3)()
        self._enter()
        check(lib().lbm_wall_force(self._h, F), "lbm_wall_force")
        return [F[0], F[1], F[2]]

    # -- discrete adjoint ----------------------------------------------------
    @property
    def buffer_bytes(self):
        return lib().lbm_buffer_bytes(self._h)

    def forward_record(self, n, k, ckpt=None):
        """Advances n steps, keeping the state every k steps; returns the
        checkpoint tensor (n/k buffers) that adjoint() needs."""
        if ckpt is None:
            ckpt = torch.empty(max(n // k, 1) * self.buffer_bytes, dtype=torch.uint8,
                               device=self.device)
        self._enter(ckpt)
        check(lib().lbm_forward_record(self._h, int(n), int(k), _ptr(ckpt)), "lbm_forward_record")
        self._leave()
        return ckpt

    def adjoint(self, n, k, ckpt, u0, dJ_du, work=None, rho0=None):
        """(dJ/du0 [3,nz,ny,nx] FP64, dJ/dtau, dJ/dF [3]) of a functional of the
        final velocity, given dJ/du^n; u0 (and, in the compressible model,
        rho0) are the fields the run started from."""
        u0 = _dev_f64(u0, (3,) + self.shape, self.device)
        rho0 = _dev_f64(rho0, self.shape, self.device)
        dJ_du = _dev_f64(dJ_du, (3,) + self.shape, self.device)
        if work is None:
            work = torch.empty(lib().lbm_adjoint_workspace_bytes(self._h, int(k)), dtype=torch.uint8,
                               device=self.device)
        u0bar = torch.empty((3,) + self.shape, dtype=torch.float64, device=self.device)
        taubar = ctypes.c_double()
        Fbar = (ctypes.c_double * 3)()
        self._enter(ckpt, work, rho0, u0, dJ_du, u0bar)
        check(lib().lbm_adjoint(self._h, int(n), int(k), _ptr(ckpt), _ptr(work), _ptr(rho0),
                                _ptr(u0), _ptr(dJ_du), _ptr(u0bar), ctypes.byref(taubar), Fbar),
              "lbm_adjoint")
        self._leave()
        return u0bar, taubar.value, [Fbar[0], Fbar[1], Fbar[2]]

    def reduce(self):
        """Monitor: {'mass', 'ke', 'umax'} in FP64 (synchronises the stream)."""
        m, k, um = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        self._enter()
        st = lib().lbm_reduce(self._h, ctypes.byref(m), ctypes.byref(k), ctypes.byref(um))
        out = {"mass": m.value, "ke": k.value, "umax": um.value,
               "unstable": st == EUNSTABLE}
        if st not in (OK, EUNSTABLE):
            check(st, "lbm_reduce")
        return out

    def reduce_noalloc(self, result):
        """Monitor into ``result`` (FP64 device tensor of 4: mass, kinetic
        energy, max |u|, non-finite count), asynchronously on the stream;
        allocates nothing (lbm_reduce_noalloc)."""
        if result.dtype != torch.float64 or not result.is_cuda or not result.is_contiguous():
            raise ValueError("result must be a contiguous FP64 device tensor")
        self._enter(result)
        check(lib().lbm_reduce_noalloc(self._h, _ptr(result)), "lbm_reduce_noalloc")
        self._leave()


class LBMRollout(torch.autograd.Function):
    """u^n = rollout(u0, tau, F): n LBM steps from f^0 = feq(rho, u0) (+ noise),
    differentiable in u0, tau and F through the library's discrete adjoint
    with checkpoints every k steps (the backward recomputes each k-step
    segment from its checkpoint).

    Call as ``LBMRollout.apply(u0, tau, force, rho, n, k, lattice, bc, storage,
    noise, compressible)`` with u0 a [3, nz, ny, nx] FP64 CUDA tensor, tau a
    scalar tensor, force a 3-vector tensor.  Returns u^n [3, nz, ny, nx]
    (FP64).
    """

    @staticmethod
    def forward(ctx, u0, tau, force, rho, n, k, lattice=D3Q19, bc=(0, 0, 0), storage="f64",
                noise=None, compressible=False):
        nz, ny, nx = u0.shape[1:]
        sim = LBM(lattice, nx, ny, nz, float(tau), force=tuple(float(v) for v in force.reshape(-1)),
                  bc=bc, storage=storage, device=u0.device, compressible=compressible)
        u0d = u0.detach().to(torch.float64).contiguous()
        rhod = _dev_f64(rho, (nz, ny, nx), u0.device)
        sim.init_equilibrium(rhod, u0d, noise)
        ckpt = sim.forward_record(n, k)
        _, uN = sim.moments()
        ctx.sim, ctx.ckpt, ctx.n, ctx.k = sim, ckpt, n, k
        ctx.tau_like, ctx.force_like = tau, force
        ctx.save_for_backward(u0d, rhod)
        return uN

    @staticmethod
    def backward(ctx, grad_u):
        u0d, rhod = ctx.saved_tensors
        u0bar, taubar, Fbar = ctx.sim.adjoint(ctx.n, ctx.k, ctx.ckpt, u0d, grad_u.contiguous(),
                                              rho0=rhod)
        ctx.sim.close()
        ctx.ckpt = None
        gt = torch.tensor(taubar, dtype=ctx.tau_like.dtype, device=ctx.tau_like.device)
        gF = torch.tensor(Fbar, dtype=ctx.force_like.dtype, device=ctx.force_like.device)
        return (u0bar, gt.reshape(ctx.tau_like.shape), gF.reshape(ctx.force_like.shape),
                None, None, None, None, None, None, None, None)
