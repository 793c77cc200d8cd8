"""ctypes binding of liblsop.so (argument marshalling only).

Every numerical step runs in the HIP library; this module checks tensor
shapes/dtypes, passes raw device pointers and the current HIP stream, and
turns status codes into exceptions.  torch supplies device memory and
streams.  Importing this module does not load the library; the first call
does, and raises if ``liblsop.so`` has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblsop.so")

# status codes (include/lsop.h)
OK, EINVAL, ENOMEM, EHIP, NOT_CONVERGED, DIVERGED, ESINGULAR, EUNSUPPORTED = range(8)
STATUS_NAMES = {OK: "OK", EINVAL: "EINVAL", ENOMEM: "ENOMEM", EHIP: "EHIP", NOT_CONVERGED: "NOT_CONVERGED",
                DIVERGED: "DIVERGED", ESINGULAR: "ESINGULAR", EUNSUPPORTED: "EUNSUPPORTED"}
C64, C128, MIXED = 0, 1, 2
MODES = {"A": 0, "G0V": 1, "AH": 2, "VHG0H": 3}
PC_IDENTITY, PC_LOWRANK, PC_HODLR, PC_SCALAR, PC_GAMMA = 0, 1, 2, 3, 4
INIT = {"h_rhs": 0, "zero": 1, "user": 2, "best": 3}

EXPORTS = ("lsop_create", "lsop_set_problem", "lsop_apply", "lsop_residual", "lsop_incident", "lsop_autotune",
           "lsop_kernel_table", "lsop_info", "lsop_destroy", "lsop_last_error", "lsop_state_bytes",
           "lsop_create_in", "lsop_workspace_bytes", "lsop_attach_workspace", "lsop_alloc_count", "lsop_apply_noalloc", "gmres_solve", "gmres_workspace_bytes", "lsop_sweep", "lsop_set_problem_damped", "lsop_bessel_host_c", "lsop_create3d",
           "lsop_set_problem3d", "lsop_incident3d",
           "precond_state_bytes", "precond_create_in", "precond_create",
           "precond_build", "precond_build_batch", "precond_apply", "precond_info", "precond_depth", "precond_destroy",
           "series_solve", "series_solve_sources", "series_sources_workspace_bytes",
           "lsop_bessel_host", "lsop_profile_enable", "lsop_profile_reset", "lsop_profile_read",
           "lsop_profile_read_kernels", "lsop_batch_create", "lsop_batch_apply", "lsop_batch_autotune",
           "lsop_batch_solve", "lsop_batch_info", "lsop_batch_destroy", "unet_create", "unet_param_count",
           "unet_set_params", "unet_init_params", "unet_get_params", "unet_forward", "unet_backward", "unet_get_grads", "unet_train_step",
           "unet_pack_inputs", "unet_pack_target", "unet_warm_start", "unet_info", "unet_destroy")


class LsopError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class OpInfo(C.Structure):
    _fields_ = [("nx", C.c_int), ("nz", C.c_int), ("lx", C.c_int), ("lz", C.c_int), ("dtype", C.c_int),
                ("max_vec", C.c_int), ("state_bytes", C.c_size_t), ("col_tile", C.c_int), ("ny", C.c_int),
                ("ly", C.c_int)]


class PrecondParams(C.Structure):
    _fields_ = [("kind", C.c_int), ("rank", C.c_int), ("power_iters", C.c_int), ("seed", C.c_uint64),
                ("levels", C.c_int), ("oversample", C.c_int), ("alpha", C.c_double), ("q_from_level", C.c_int),
                ("min_width", C.c_int)]


class SolveParams(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int), ("init", C.c_int), ("refine_max", C.c_int),
                ("inner_tol", C.c_double)]


class GmresParams(C.Structure):
    _fields_ = [("tol", C.c_double), ("restart", C.c_int), ("max_iter", C.c_int), ("init", C.c_int),
                ("refine_max", C.c_int), ("inner_tol", C.c_double)]


class SweepParams(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int), ("escalate_above", C.c_int), ("rank_step", C.c_int),
                ("rank_max", C.c_int), ("max_rebuilds", C.c_int), ("ricker_fc", C.c_double)]


class SweepInfo(C.Structure):
    _fields_ = [("freq", C.c_double), ("rank", C.c_int), ("rebuilds", C.c_int), ("iters_max", C.c_int),
                ("status", C.c_int), ("rel_residual_max", C.c_double)]


class KernelStat(C.Structure):
    _fields_ = [("name", C.c_char * 48), ("launches", C.c_int), ("total_ms", C.c_double), ("bytes", C.c_double),
                ("flops", C.c_double), ("items", C.c_double)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("refine_steps", C.c_int), ("rel_residual", C.c_double), ("status", C.c_int),
                ("rel_residual0", C.c_double)]


_lib = None


def load_library(path=LIB_PATH):
    """Load liblsop.so and declare its signatures (no GPU call is made)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2005_01372_amd.build`")
    lib = C.CDLL(path)
    vp, ip, dp = C.c_void_p, C.c_int, C.c_double
    sig = {
        "lsop_create": (ip, [ip, ip, ip, ip, C.POINTER(vp)]),
        "lsop_set_problem": (ip, [vp, vp, dp, dp, dp, vp]),
        "lsop_apply": (ip, [vp, ip, vp, vp, ip, vp]),
        "lsop_set_problem_damped": (ip, [vp, vp, dp, dp, dp, dp, ip, vp]),
        "lsop_bessel_host_c": (ip, [ip, dp, dp, C.POINTER(dp)]),
        "lsop_create3d": (ip, [ip, ip, ip, ip, ip, C.POINTER(vp)]),
        "lsop_set_problem3d": (ip, [vp, vp, dp, dp, dp, vp]),
        "lsop_incident3d": (ip, [vp, vp, vp, ip, vp, vp]),
        "lsop_residual": (ip, [vp, vp, vp, vp, vp, ip, vp]),
        "lsop_incident": (ip, [vp, vp, vp, vp, ip, vp, vp]),
        "lsop_kernel_table": (ip, [vp, vp, vp]),
        "lsop_autotune": (ip, [vp, ip, vp]),
        "lsop_info": (ip, [vp, C.POINTER(OpInfo)]),
        "lsop_destroy": (None, [vp]),
        "lsop_last_error": (C.c_char_p, []),
        "lsop_state_bytes": (ip, [ip, ip, ip, ip, C.POINTER(C.c_size_t)]),
        "lsop_create_in": (ip, [ip, ip, ip, ip, vp, C.c_size_t, C.POINTER(vp)]),
        "lsop_workspace_bytes": (ip, [vp, ip, ip, C.POINTER(C.c_size_t)]),
        "lsop_attach_workspace": (ip, [vp, vp, C.c_size_t]),
        "lsop_alloc_count": (ip, [C.POINTER(C.c_size_t)]),
        "lsop_apply_noalloc": (ip, [vp, ip, vp, vp, ip, vp]),
        "gmres_solve": (ip, [vp, vp, vp, vp, ip, C.POINTER(GmresParams), C.POINTER(SolveInfo), vp]),
        "gmres_workspace_bytes": (ip, [vp, ip, ip, C.POINTER(C.c_size_t)]),
        "lsop_sweep": (ip, [vp, vp, dp, dp, C.POINTER(dp), ip, C.POINTER(PrecondParams), C.POINTER(SweepParams),
                            vp, vp, ip, vp, C.POINTER(SweepInfo), vp]),
        "precond_state_bytes": (ip, [vp, C.POINTER(PrecondParams), C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
        "precond_create_in": (ip, [vp, C.POINTER(PrecondParams), vp, C.c_size_t, C.POINTER(vp)]),
        "precond_create": (ip, [vp, C.POINTER(PrecondParams), C.POINTER(vp)]),
        "precond_build": (ip, [vp, vp, vp]),
        "precond_build_batch": (ip, [vp, C.c_int, C.c_int]),
        "precond_apply": (ip, [vp, vp, vp, ip, vp]),
        "precond_info": (ip, [vp, C.POINTER(ip), C.POINTER(dp), C.POINTER(C.c_size_t)]),
        "precond_depth": (ip, [vp, C.POINTER(ip)]),
        "precond_destroy": (None, [vp]),
        "series_solve": (ip, [vp, vp, vp, vp, ip, C.POINTER(SolveParams), C.POINTER(SolveInfo), vp]),
        "series_solve_sources": (ip, [vp, vp, vp, vp, vp, ip, vp, C.POINTER(SolveParams), C.POINTER(SolveInfo), vp]),
        "series_sources_workspace_bytes": (ip, [vp, ip, ip, C.POINTER(C.c_size_t)]),
        "lsop_bessel_host": (ip, [ip, dp, C.POINTER(dp)]),
        "lsop_profile_enable": (ip, [ip]),
        "lsop_profile_reset": (ip, []),
        "lsop_profile_read": (ip, [C.POINTER(KernelStat), ip, C.POINTER(ip)]),
        "lsop_profile_read_kernels": (ip, [C.POINTER(KernelStat), ip, C.POINTER(ip)]),
        "lsop_batch_create": (ip, [ip, C.POINTER(vp), C.POINTER(vp)]),
        "lsop_batch_apply": (ip, [vp, ip, C.POINTER(vp), C.POINTER(vp), C.POINTER(ip), vp]),
        "lsop_batch_autotune": (ip, [vp, vp]),
        "lsop_batch_solve": (ip, [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), C.POINTER(ip),
                                  C.POINTER(SolveParams), ip, C.POINTER(SolveInfo), vp]),
        "lsop_batch_info": (ip, [vp, C.POINTER(ip), C.POINTER(C.c_size_t)]),
        "lsop_batch_destroy": (None, [vp]),
        "unet_create": (ip, [ip, ip, ip, ip, ip, ip, ip, C.POINTER(vp)]),
        "unet_param_count": (ip, [vp, C.POINTER(C.c_size_t)]),
        "unet_set_params": (ip, [vp, vp, vp]),
        "unet_get_params": (ip, [vp, vp, vp]),
        "unet_init_params": (ip, [vp, C.c_ulonglong, vp]),
        "unet_forward": (ip, [vp, vp, ip, ip, ip, vp, vp]),
        "unet_backward": (ip, [vp, vp, vp]),
        "unet_get_grads": (ip, [vp, vp, vp]),
        "unet_train_step": (ip, [vp, vp, vp, ip, ip, ip, C.c_float, C.POINTER(dp), vp]),
        "unet_pack_inputs": (ip, [vp, vp, vp, ip, vp, vp, vp]),
        "unet_pack_target": (ip, [vp, vp, vp, vp, ip, vp, vp]),
        "unet_warm_start": (ip, [vp, vp, vp, vp, ip, vp]),
        "unet_info": (ip, [vp, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
        "unet_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(status, allow=()):
    if status != OK and status not in allow:
        raise LsopError(status, _lib.lsop_last_error().decode())
    return status


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _gpu(*tensors):
    """Raise unless every tensor lives on the GPU (called after the shape and dtype checks of a call)."""
    for t in tensors:
        if not t.is_cuda:
            raise TypeError("tensors passed to the library must be on the GPU")


def bessel_host(kind, x):
    lib = load_library()
    out = (C.c_double * 2)()
    _check(lib.lsop_bessel_host(int(kind), float(x), out))
    return out[0], out[1]


def state_bytes(nx, nz, dtype=C128, max_vec=64):
    """Device bytes of an operator's state (lsop_state_bytes; host only)."""
    b = C.c_size_t()
    _check(load_library().lsop_state_bytes(int(nx), int(nz), int(dtype), int(max_vec), C.byref(b)))
    return b.value


def alloc_count():
    """Device allocations the library has made in this process (lsop_alloc_count)."""
    c = C.c_size_t()
    _check(load_library().lsop_alloc_count(C.byref(c)))
    return c.value


def _byte_buffer(t, need, what):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous()):
        raise TypeError(f"{what} must be a contiguous CUDA tensor")
    if t.numel() * t.element_size() < need:
        raise ValueError(f"{what} holds {t.numel() * t.element_size()} bytes, {need} needed")
    if t.data_ptr() % 256:
        raise ValueError(f"{what} must be 256-byte aligned")
    return t


def bessel_host_c(kind, z):
    """Host evaluation of the library's complex-argument Bessel routines: kind 0 -> H0^(1)(z); kind 1 -> (J1, Y1)."""
    lib = load_library()
    out = (C.c_double * 4)()
    _check(lib.lsop_bessel_host_c(int(kind), float(complex(z).real), float(complex(z).imag), out))
    if kind == 0:
        return complex(out[0], out[1])
    return complex(out[0], out[1]), complex(out[2], out[3])


def profile_enable(on=True):
    _check(load_library().lsop_profile_enable(int(bool(on))))


def profile_reset():
    _check(load_library().lsop_profile_reset())


def profile_read(by_kernel=False):
    """Totals since the last reset, by use label or (by_kernel) by kernel function:
    {name: dict(launches, ms, bytes, flops, items)}."""
    lib = load_library()
    arr = (KernelStat * 128)()
    cnt = C.c_int()
    fn = lib.lsop_profile_read_kernels if by_kernel else lib.lsop_profile_read
    _check(fn(arr, 128, C.byref(cnt)))
    return {arr[i].name.decode(): dict(launches=arr[i].launches, ms=arr[i].total_ms, bytes=arr[i].bytes,
                                       flops=arr[i].flops, items=arr[i].items) for i in range(min(cnt.value, 128))}


class Operator:
    """The LS operator of one grid and medium (lsop_create + lsop_set_problem).

    state: optional caller-owned device buffer (a CUDA tensor of at least state_bytes(...) bytes) that holds the
    operator's device state instead of library allocations (lsop_create_in); it is kept alive by the object."""

    def __init__(self, nx, nz, dtype=C128, max_vec=64, state=None):
        self.lib = load_library()
        self.nx, self.nz, self.dtype, self.max_vec = int(nx), int(nz), int(dtype), int(max_vec)
        h = C.c_void_p()
        if state is None:
            _check(self.lib.lsop_create(self.nx, self.nz, self.dtype, self.max_vec, C.byref(h)))
        else:
            need = state_bytes(self.nx, self.nz, self.dtype, self.max_vec)
            self._state = _byte_buffer(state, need, "state")
            _check(self.lib.lsop_create_in(self.nx, self.nz, self.dtype, self.max_vec, _ptr(state),
                                           state.numel() * state.element_size(), C.byref(h)))
        self.handle = h
        self.vec_dtype = torch.complex64 if self.dtype == C64 else torch.complex128
        self.inner_dtype = torch.complex64 if self.dtype in (C64, MIXED) else torch.complex128

    def close(self):
        if getattr(self, "handle", None):
            self.lib.lsop_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        inf = OpInfo()
        _check(self.lib.lsop_info(self.handle, C.byref(inf)))
        return inf

    def set_problem(self, vel, h, freq, c0=2000.0):
        vel = torch.as_tensor(vel, dtype=torch.float64)
        if not vel.is_cuda:
            vel = vel.cuda()
        vel = vel.contiguous()
        if tuple(vel.shape) != (self.nx, self.nz):
            raise ValueError(f"velocity must be {(self.nx, self.nz)}")
        self._vel = vel
        _check(self.lib.lsop_set_problem(self.handle, _ptr(vel), float(h), float(freq), float(c0), _stream()))
        self.h, self.freq, self.c0 = float(h), float(freq), float(c0)
        return self

    def set_problem_damped(self, vel, h, freq, c0=2000.0, eps=None, absorb=0):
        """The convergent Born series' medium (lsop_set_problem_damped): dissipative background k0^2 + i eps, gain
        in the potential, optional absorbing layer of `absorb` cells."""
        vel = torch.as_tensor(vel, dtype=torch.float64)
        if not vel.is_cuda:
            vel = vel.cuda()
        vel = vel.contiguous()
        if tuple(vel.shape) != (self.nx, self.nz):
            raise ValueError(f"velocity must be {(self.nx, self.nz)}")
        self._vel = vel
        _check(self.lib.lsop_set_problem_damped(self.handle, _ptr(vel), float(h), float(freq), float(c0), float(eps),
                                                int(absorb), _stream()))
        self.h, self.freq, self.c0, self.eps = float(h), float(freq), float(c0), float(eps)
        return self

    def _vecs(self, x, dtype=None, nvec=None):
        """Number of [nx][nz] vectors in x, after checking its shape, dtype, layout and device (and, when
        nvec is given, that it holds exactly that many vectors)."""
        dtype = dtype or self.vec_dtype
        if not isinstance(x, torch.Tensor):
            raise TypeError("expected a torch tensor")
        if x.dim() < 2 or tuple(x.shape[-2:]) != (self.nx, self.nz):
            raise ValueError(f"vectors must end in {(self.nx, self.nz)}, got {tuple(x.shape)}")
        nv = x.numel() // (self.nx * self.nz)
        if nvec is not None and nv != nvec:
            raise ValueError(f"expected {nvec} vectors, got {nv}")
        if x.dtype != dtype:
            raise TypeError(f"expected {dtype}, got {x.dtype}")
        if not x.is_contiguous():
            raise ValueError("vectors must be contiguous")
        return nv

    def apply(self, x, mode="A", out=None):
        nv = self._vecs(x)
        out = torch.empty_like(x) if out is None else out
        self._vecs(out, nvec=nv)
        _gpu(x, out)
        _check(self.lib.lsop_apply(self.handle, MODES[mode], _ptr(x), _ptr(out), nv, _stream()))
        return out

    def apply_noalloc(self, x, mode="A", out=None):
        """lsop_apply_noalloc: as apply, with the FFT intermediate in the library's fixed device array (no
        device allocation by the library; out must then be supplied to avoid torch's)."""
        nv = self._vecs(x)
        out = torch.empty_like(x) if out is None else out
        self._vecs(out, nvec=nv)
        _gpu(x, out)
        _check(self.lib.lsop_apply_noalloc(self.handle, MODES[mode], _ptr(x), _ptr(out), nv, _stream()))
        return out

    def residual(self, psi, rhs, out=None):
        nv = self._vecs(psi)
        self._vecs(rhs, nvec=nv)
        out = torch.empty_like(psi) if out is None else out
        self._vecs(out, nvec=nv)
        _gpu(psi, rhs, out)
        nrm = torch.empty(nv, dtype=torch.float64, device=psi.device)
        _check(self.lib.lsop_residual(self.handle, _ptr(psi), _ptr(rhs), _ptr(out), _ptr(nrm), nv, _stream()))
        return out, nrm

    @staticmethod
    def _sources(src_i, src_j, amp):
        if len(src_i) != len(src_j) or (amp is not None and len(amp) != len(src_i)):
            raise ValueError("src_i, src_j (and amp) must have one entry per source")
        si = (C.c_int * len(src_i))(*[int(v) for v in src_i])
        sj = (C.c_int * len(src_j))(*[int(v) for v in src_j])
        if amp is not None:
            a = []
            for v in amp:
                a += [complex(v).real, complex(v).imag]
            ap = (C.c_double * len(a))(*a)
        else:
            ap = None
        return si, sj, ap

    def incident(self, src_i, src_j, amp=None):
        si, sj, ap = self._sources(src_i, src_j, amp)
        out = torch.empty((len(src_i), self.nx, self.nz), dtype=self.vec_dtype, device="cuda")
        _check(self.lib.lsop_incident(self.handle, si, sj, ap, len(src_i), _ptr(out), _stream()))
        return out

    def workspace_bytes(self, nvec, init="h_rhs"):
        """Workspace that set_problem and a series on nvec right-hand sides need (lsop_workspace_bytes)."""
        b = C.c_size_t()
        _check(self.lib.lsop_workspace_bytes(self.handle, int(nvec), INIT[init], C.byref(b)))
        return b.value

    def attach_workspace(self, ws):
        """Hand the operator a caller-owned workspace (a CUDA tensor; None returns to library-owned growth)."""
        if ws is None:
            _check(self.lib.lsop_attach_workspace(self.handle, None, 0))
        else:
            _byte_buffer(ws, 1, "workspace")
            _check(self.lib.lsop_attach_workspace(self.handle, _ptr(ws), ws.numel() * ws.element_size()))
        self._ws = ws

    def autotune(self, nvec):
        """Pick the fastest column-pass tile for batches of nvec vectors; returns the chosen width."""
        _check(self.lib.lsop_autotune(self.handle, int(nvec), _stream()))
        return self.info().col_tile

    def kernel_table(self):
        out = torch.empty((self.nx, self.nz), dtype=torch.complex128, device="cuda")
        _check(self.lib.lsop_kernel_table(self.handle, _ptr(out), _stream()))
        return out


class Operator3D(Operator):
    """The 3D LS operator (lsop_create3d + lsop_set_problem3d); vectors [..][nx][ny][nz].  Series, GMRES and
    the low-rank / scalar preconditioners take it like a 2D operator."""

    def __init__(self, nx, ny, nz, dtype=C128, max_vec=16):
        self.lib = load_library()
        self.nx, self.ny, self.nz, self.dtype, self.max_vec = int(nx), int(ny), int(nz), int(dtype), int(max_vec)
        h = C.c_void_p()
        _check(self.lib.lsop_create3d(self.nx, self.ny, self.nz, self.dtype, self.max_vec, C.byref(h)))
        self.handle = h
        self.vec_dtype = torch.complex64 if self.dtype == C64 else torch.complex128
        self.inner_dtype = torch.complex64 if self.dtype in (C64, MIXED) else torch.complex128

    def set_problem(self, vel, h, freq, c0=2000.0):
        vel = torch.as_tensor(vel, dtype=torch.float64)
        vel = (vel if vel.is_cuda else vel.cuda()).contiguous()
        if tuple(vel.shape) != (self.nx, self.ny, self.nz):
            raise ValueError(f"velocity must be {(self.nx, self.ny, self.nz)}")
        self._vel = vel
        _check(self.lib.lsop_set_problem3d(self.handle, _ptr(vel), float(h), float(freq), float(c0), _stream()))
        self.h, self.freq, self.c0 = float(h), float(freq), float(c0)
        return self

    def _vecs(self, x, dtype=None, nvec=None):
        dtype = dtype or self.vec_dtype
        if not isinstance(x, torch.Tensor):
            raise TypeError("expected a torch tensor")
        if x.dim() < 3 or tuple(x.shape[-3:]) != (self.nx, self.ny, self.nz):
            raise ValueError(f"vectors must end in {(self.nx, self.ny, self.nz)}, got {tuple(x.shape)}")
        nv = x.numel() // (self.nx * self.ny * self.nz)
        if nvec is not None and nv != nvec:
            raise ValueError(f"expected {nvec} vectors, got {nv}")
        if x.dtype != dtype:
            raise TypeError(f"expected {dtype}, got {x.dtype}")
        if not x.is_contiguous():
            raise ValueError("vectors must be contiguous")
        return nv

    def incident(self, src, amp=None):
        src = [tuple(int(v) for v in s) for s in src]
        flat = (C.c_int * (3 * len(src)))(*[v for s in src for v in s])
        if amp is not None:
            a = []
            for v in amp:
                a += [complex(v).real, complex(v).imag]
            ap = (C.c_double * len(a))(*a)
        else:
            ap = None
        out = torch.empty((len(src), self.nx, self.ny, self.nz), dtype=self.vec_dtype, device="cuda")
        _check(self.lib.lsop_incident3d(self.handle, flat, ap, len(src), _ptr(out), _stream()))
        return out

    def kernel_table(self):
        out = torch.empty((self.nx, self.ny, self.nz), dtype=torch.complex128, device="cuda")
        _check(self.lib.lsop_kernel_table(self.handle, _ptr(out), _stream()))
        return out


class Preconditioner:
    """H for the series: identity (Born), the randomized low-rank SMW form (Alg. 2 + eq. 12), or the
    inverse of the HODLR approximation of I - G0 V (Section 2.4, ``levels`` tree levels)."""

    def __init__(self, op, kind=PC_LOWRANK, rank=32, power_iters=0, seed=0, levels=0, oversample=0, alpha=0.0,
                 state=None, q_from_level=0, min_width=0):
        self.op, self.lib = op, op.lib
        p = PrecondParams(int(kind), int(rank), int(power_iters), int(seed), int(levels), int(oversample),
                          float(alpha), int(q_from_level), int(min_width))
        h = C.c_void_p()
        if state is None:
            _check(self.lib.precond_create(op.handle, C.byref(p), C.byref(h)))
        else:
            need, _ = Preconditioner.state_bytes(op, kind, rank, power_iters, seed, levels, oversample, alpha,
                                                 q_from_level, min_width)
            self._state = _byte_buffer(state, need, "state")
            _check(self.lib.precond_create_in(op.handle, C.byref(p), _ptr(state), state.numel() * state.element_size(),
                                              C.byref(h)))
        self.handle = h
        depth = C.c_int()
        _check(self.lib.precond_depth(h, C.byref(depth)))
        # HODLR: the tree depth after the minimum-width rule (the number of probe blocks build() takes)
        self.kind, self.rank, self.levels, self.oversample = kind, rank, depth.value or levels, oversample

    @staticmethod
    def state_bytes(op, kind=PC_LOWRANK, rank=32, power_iters=0, seed=0, levels=0, oversample=0, alpha=0.0,
                    q_from_level=0, min_width=0):
        """(state bytes, build workspace bytes) of a preconditioner of `op` (precond_state_bytes; host only)."""
        p = PrecondParams(int(kind), int(rank), int(power_iters), int(seed), int(levels), int(oversample),
                          float(alpha), int(q_from_level), int(min_width))
        st, ws = C.c_size_t(), C.c_size_t()
        _check(op.lib.precond_state_bytes(op.handle, C.byref(p), C.byref(st), C.byref(ws)))
        return st.value, ws.value

    def close(self):
        if getattr(self, "handle", None):
            self.lib.precond_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def build(self, omega=None):
        if omega is not None:
            omega = torch.as_tensor(omega, dtype=torch.float64)
            omega = (omega if omega.is_cuda else omega.cuda()).contiguous()
            blocks = self.levels if self.kind == PC_HODLR else 1
            if omega.numel() != blocks * (self.rank + self.oversample) * self.op.nx * self.op.nz:
                raise ValueError("omega must hold (levels x) (rank + oversample) x nx*nz values")
            self._omega = omega
        return _check(self.lib.precond_build(self.handle, _ptr(omega) if omega is not None else None, _stream()))

    def apply(self, x, out=None):
        nv = self.op._vecs(x, self.op.inner_dtype)
        out = torch.empty_like(x) if out is None else out
        self.op._vecs(out, self.op.inner_dtype, nvec=nv)
        _gpu(x, out)
        _check(self.lib.precond_apply(self.handle, _ptr(x), _ptr(out), nv, _stream()))
        return out

    def info(self):
        r, comp, nb = C.c_int(), C.c_double(), C.c_size_t()
        _check(self.lib.precond_info(self.handle, C.byref(r), C.byref(comp), C.byref(nb)))
        return r.value, comp.value, nb.value


@dataclass
class SolveResult:
    iters: int
    refine_steps: int
    rel_residual: float
    status: int
    rel_residual0: float

    @property
    def status_name(self):
        return STATUS_NAMES.get(self.status, str(self.status))


def series_solve(op, pc, rhs, psi=None, tol=1e-10, max_iter=30, init="h_rhs", refine_max=8, inner_tol=1e-5,
                 raise_on_failure=False):
    """Preconditioned scattering series (eq. 11); returns (psi, [SolveResult per right-hand side])."""
    nv = op._vecs(rhs)
    psi = torch.empty_like(rhs) if psi is None else psi
    op._vecs(psi, nvec=nv)
    _gpu(rhs, psi)
    p = SolveParams(float(tol), int(max_iter), INIT[init], int(refine_max), float(inner_tol))
    info = (SolveInfo * nv)()
    st = op.lib.series_solve(op.handle, pc.handle if pc is not None else None, _ptr(rhs), _ptr(psi), nv,
                             C.byref(p), info, _stream())
    _check(st, allow=() if raise_on_failure else (NOT_CONVERGED, DIVERGED))
    return psi, [SolveResult(i.iters, i.refine_steps, i.rel_residual, i.status, i.rel_residual0) for i in info]


def series_solve_sources(op, pc, src_i, src_j, amp=None, psi=None, tol=1e-10, max_iter=30, init="h_rhs",
                         refine_max=8, inner_tol=1e-5, raise_on_failure=False):
    """The series for point sources (series_solve_sources): the incident fields are formed in the operator's
    workspace; returns (psi, [SolveResult per source])."""
    si, sj, ap = op._sources(src_i, src_j, amp)
    ns = len(src_i)
    if ns < 1:
        raise ValueError("at least one source")
    psi = torch.empty((ns, op.nx, op.nz), dtype=op.vec_dtype, device="cuda") if psi is None else psi
    op._vecs(psi, nvec=ns)
    _gpu(psi)
    p = SolveParams(float(tol), int(max_iter), INIT[init], int(refine_max), float(inner_tol))
    info = (SolveInfo * ns)()
    st = op.lib.series_solve_sources(op.handle, pc.handle if pc is not None else None, si, sj, ap, ns, _ptr(psi),
                                     C.byref(p), info, _stream())
    _check(st, allow=() if raise_on_failure else (NOT_CONVERGED, DIVERGED))
    return psi, [SolveResult(i.iters, i.refine_steps, i.rel_residual, i.status, i.rel_residual0) for i in info]


def series_sources_workspace_bytes(op, nsrc, init="h_rhs"):
    """Workspace of series_solve_sources for nsrc sources (host only)."""
    b = C.c_size_t()
    _check(op.lib.series_sources_workspace_bytes(op.handle, int(nsrc), INIT[init], C.byref(b)))
    return b.value


def gmres_solve(op, pc, rhs, psi=None, tol=1e-10, restart=30, max_iter=300, init="zero", refine_max=8,
                inner_tol=1e-5, raise_on_failure=False):
    """Restarted GMRES(restart), right-preconditioned by pc (Section 3.2.3's comparison method); returns
    (psi, [SolveResult per right-hand side]) with iters = inner iterations."""
    nv = op._vecs(rhs)
    psi = torch.empty_like(rhs) if psi is None else psi
    op._vecs(psi, nvec=nv)
    _gpu(rhs, psi)
    p = GmresParams(float(tol), int(restart), int(max_iter), INIT[init], int(refine_max), float(inner_tol))
    info = (SolveInfo * nv)()
    st = op.lib.gmres_solve(op.handle, pc.handle if pc is not None else None, _ptr(rhs), _ptr(psi), nv,
                            C.byref(p), info, _stream())
    _check(st, allow=() if raise_on_failure else (NOT_CONVERGED, DIVERGED))
    return psi, [SolveResult(i.iters, i.refine_steps, i.rel_residual, i.status, i.rel_residual0) for i in info]


def sweep(op, vel, h, c0, freqs, src_i, src_j, kind=PC_LOWRANK, rank=8, levels=0, power_iters=0, oversample=0,
          seed=0, tol=1e-6, max_iter=30, escalate_above=10, rank_step=8, rank_max=256, max_rebuilds=8,
          ricker_fc=0.0):
    """Frequency sweep of Section 3.1 (lowest first, rank escalation, restart from psi0); returns
    (psi [nfreq][nsrc][nx][nz], [dict per frequency])."""
    vel = torch.as_tensor(vel, dtype=torch.float64)
    vel = (vel if vel.is_cuda else vel.cuda()).contiguous()
    if tuple(vel.shape) != (op.nx, op.nz):
        raise ValueError(f"velocity must be {(op.nx, op.nz)}")
    nf, ns = len(freqs), len(src_i)
    if len(src_j) != ns:
        raise ValueError("src_i and src_j differ in length")
    f = (C.c_double * nf)(*[float(v) for v in freqs])
    si = (C.c_int * ns)(*[int(v) for v in src_i])
    sj = (C.c_int * ns)(*[int(v) for v in src_j])
    pp = PrecondParams(int(kind), int(rank), int(power_iters), int(seed), int(levels), int(oversample), 0.0)
    sp = SweepParams(float(tol), int(max_iter), int(escalate_above), int(rank_step), int(rank_max),
                     int(max_rebuilds), float(ricker_fc))
    psi = torch.empty((nf, ns, op.nx, op.nz), dtype=op.vec_dtype, device="cuda")
    info = (SweepInfo * nf)()
    st = op.lib.lsop_sweep(op.handle, _ptr(vel), float(h), float(c0), f, nf, C.byref(pp), C.byref(sp), si, sj, ns,
                           _ptr(psi), info, _stream())
    _check(st, allow=(NOT_CONVERGED, DIVERGED, ESINGULAR))
    op.h, op.c0, op.freq = float(h), float(c0), float(freqs[-1])
    return psi, [dict(freq=i.freq, rank=i.rank, rebuilds=i.rebuilds, iters_max=i.iters_max, status=i.status,
                      rel_residual_max=i.rel_residual_max) for i in info]


def build_batch(pcs, streams=4):
    """Builds several preconditioners (distinct operators) concurrently on `streams` device streams."""
    pcs = list(pcs)
    arr = (C.c_void_p * max(1, len(pcs)))(*[pc.handle for pc in pcs])
    return _check(load_library().precond_build_batch(arr, len(pcs), int(streams)))


class Batch:
    """Instances of uneven size advanced together: one launch per FFT pass per grid-shape group."""

    def __init__(self, ops):
        self.ops = list(ops)
        self.lib = self.ops[0].lib
        arr = (C.c_void_p * len(self.ops))(*[op.handle.value for op in self.ops])
        h = C.c_void_p()
        _check(self.lib.lsop_batch_create(len(self.ops), arr, C.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            self.lib.lsop_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _arrays(self, xs, dtype=None, nvec=None):
        if len(xs) != len(self.ops):
            raise ValueError("one tensor per instance")
        nvec = nvec or [None] * len(xs)
        nv = [op._vecs(x, dtype, k) for op, x, k in zip(self.ops, xs, nvec)]
        ptrs = (C.c_void_p * len(xs))(*[x.data_ptr() for x in xs])
        return ptrs, (C.c_int * len(xs))(*nv)

    def apply(self, xs, mode="A", outs=None):
        outs = [torch.empty_like(x) for x in xs] if outs is None else outs
        px, nv = self._arrays(xs)
        py, _ = self._arrays(outs, nvec=list(nv))
        _gpu(*xs, *outs)
        _check(self.lib.lsop_batch_apply(self.handle, MODES[mode], px, py, nv, _stream()))
        return outs

    def autotune(self):
        _check(self.lib.lsop_batch_autotune(self.handle, _stream()))

    def info(self):
        g, nb = C.c_int(), C.c_size_t()
        _check(self.lib.lsop_batch_info(self.handle, C.byref(g), C.byref(nb)))
        return g.value, nb.value

    def solve(self, pcs, rhss, psis=None, tol=1e-10, max_iter=30, init="h_rhs", use_graph=True):
        """Lockstep series for all instances; returns (psis, [[SolveResult per vector] per instance])."""
        psis = [torch.empty_like(r) for r in rhss] if psis is None else psis
        pr, nv = self._arrays(rhss)
        pp, _ = self._arrays(psis, nvec=list(nv))
        if len(pcs) != len(self.ops):
            raise ValueError("one preconditioner (or None) per instance")
        _gpu(*rhss, *psis)
        pch = (C.c_void_p * len(self.ops))(*[(pc.handle.value if pc is not None else None) for pc in pcs])
        total = sum(nv)
        info = (SolveInfo * max(total, 1))()
        p = SolveParams(float(tol), int(max_iter), INIT[init], 0, 0.0)
        st = self.lib.lsop_batch_solve(self.handle, pch, pr, pp, nv, C.byref(p), int(bool(use_graph)), info,
                                       _stream())
        _check(st, allow=(NOT_CONVERGED, DIVERGED))
        out, k = [], 0
        for n in nv:
            out.append([SolveResult(i.iters, i.refine_steps, i.rel_residual, i.status, i.rel_residual0)
                        for i in info[k:k + n]])
            k += n
        return psis, out


class UNet:
    """Convolutional warm start of the series (bf16 matrix-core convolutions, FP32 master weights, Adam)."""

    def __init__(self, levels=4, base=32, cin=4, cout=2, max_batch=16, max_h=128, max_w=128):
        self.lib = load_library()
        h = C.c_void_p()
        _check(self.lib.unet_create(levels, base, cin, cout, max_batch, max_h, max_w, C.byref(h)))
        self.handle = h
        self.levels, self.base, self.cin, self.cout = levels, base, cin, cout
        n = C.c_size_t()
        _check(self.lib.unet_param_count(h, C.byref(n)))
        self.nparams = n.value

    def close(self):
        if getattr(self, "handle", None):
            self.lib.unet_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _f32(t, shape=None):
        if not isinstance(t, torch.Tensor):
            raise TypeError("expected a torch tensor")
        if shape is not None and tuple(t.shape) != tuple(shape):
            raise ValueError(f"expected shape {tuple(shape)}, got {tuple(t.shape)}")
        if t.dtype != torch.float32 or not t.is_contiguous():
            raise TypeError("expected a contiguous float32 tensor")
        if not t.is_cuda:
            raise TypeError("expected a tensor on the GPU")
        return t

    def set_params(self, params):
        p = torch.as_tensor(params, dtype=torch.float32)
        p = (p if p.is_cuda else p.cuda()).contiguous()
        if p.numel() != self.nparams:
            raise ValueError(f"expected {self.nparams} parameters")
        self._p = p
        _check(self.lib.unet_set_params(self.handle, _ptr(p), _stream()))

    def init_params(self, seed=0):
        """He-normal weights, zero biases (device Philox stream keyed by seed); resets the optimizer."""
        _check(self.lib.unet_init_params(self.handle, int(seed), _stream()))

    def params(self):
        out = torch.empty(self.nparams, dtype=torch.float32, device="cuda")
        _check(self.lib.unet_get_params(self.handle, _ptr(out), _stream()))
        return out

    def forward(self, x):
        if not isinstance(x, torch.Tensor) or x.dim() != 4 or x.shape[3] != self.cin:
            raise ValueError(f"input must be [B][H][W][{self.cin}]")
        self._f32(x)
        B, H, W, c = x.shape
        y = torch.empty((B, H, W, self.cout), dtype=torch.float32, device="cuda")
        self._x = x
        self._out_shape = (B, H, W, self.cout)
        _check(self.lib.unet_forward(self.handle, _ptr(x), B, H, W, _ptr(y), _stream()))
        return y

    def backward(self, dy):
        shape = getattr(self, "_out_shape", None)
        if shape is None:
            raise RuntimeError("backward needs a preceding forward")
        self._f32(dy, shape)
        _check(self.lib.unet_backward(self.handle, _ptr(dy), _stream()))
        g = torch.empty(self.nparams, dtype=torch.float32, device="cuda")
        _check(self.lib.unet_get_grads(self.handle, _ptr(g), _stream()))
        return g

    def train_step(self, x, target, lr):
        if not isinstance(x, torch.Tensor) or x.dim() != 4 or x.shape[3] != self.cin:
            raise ValueError(f"input must be [B][H][W][{self.cin}]")
        self._f32(x)
        B, H, W, _ = x.shape
        self._f32(target, (B, H, W, self.cout))
        loss = C.c_double()
        _check(self.lib.unet_train_step(self.handle, _ptr(x), _ptr(target), B, H, W, float(lr), C.byref(loss),
                                        _stream()))
        return loss.value

    def pack_inputs(self, op, psi0):
        nv = op._vecs(psi0)
        _gpu(psi0)
        x = torch.empty((nv, op.nx, op.nz, 4), dtype=torch.float32, device="cuda")
        sc = torch.empty(nv, dtype=torch.float32, device="cuda")
        _check(self.lib.unet_pack_inputs(self.handle, op.handle, _ptr(psi0), nv, _ptr(x), _ptr(sc), _stream()))
        return x, sc

    def pack_target(self, op, psi, psi0, scale):
        nv = op._vecs(psi0)
        op._vecs(psi, nvec=nv)
        self._f32(scale, (nv,))
        _gpu(psi, psi0)
        t = torch.empty((nv, op.nx, op.nz, 2), dtype=torch.float32, device="cuda")
        _check(self.lib.unet_pack_target(op.handle, _ptr(psi), _ptr(psi0), _ptr(self._f32(scale)), nv, _ptr(t),
                                         _stream()))
        return t

    def warm_start(self, op, psi0, out=None):
        nv = op._vecs(psi0)
        out = torch.empty_like(psi0) if out is None else out
        op._vecs(out, psi0.dtype, nvec=nv)
        _gpu(psi0, out)
        _check(self.lib.unet_warm_start(self.handle, op.handle, _ptr(psi0), _ptr(out), nv, _stream()))
        return out
