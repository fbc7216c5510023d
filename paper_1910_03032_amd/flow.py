"""Velocity-correction projection steps (Section 4.2) through the C ABI.

The step runs in the library (`sfem_flow_step`, include/sfem.h): equal-order velocity and
pressure, no-slip walls on the essential DoFs of the mesh, constant nu and dt, BDF-k for
the implicit terms and EXT-k for the explicit ones (k ramps up 1, 2, ... to `order` over
the first steps), the rotational form of the pressure boundary term, the pure-Neumann
pressure Poisson solve and the three-member Helmholtz solve.  This module only marshals
arguments: the BDF/EXT weights come from `sfem_bdf_ext_weights`, every arithmetic step of
the step from the library's kernels.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import FlowInfo, FlowOpts, SfemError
from . import PcgResult, check_mesh_shapes


def bdf_ext_weights(k: int):
    """(b_0..b_k, a_1..a_k) of the library's `sfem_bdf_ext_weights` (a host computation)."""
    if k not in (1, 2, 3):
        raise ValueError("order 1, 2 or 3")
    lib = _lib.load()
    b = (C.c_double * (k + 1))()
    a = (C.c_double * k)()
    st = lib.sfem_bdf_ext_weights(int(k), b, a)
    if st != 0:
        raise SfemError(st, "sfem_bdf_ext_weights")
    return np.array(b[:], dtype=np.float64), np.array(a[:], dtype=np.float64)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else None


class ProjectionStepper:
    """Projection time stepping on one mesh (a library `sfem_flow` object).

    elem_xyz [nelem, 8, 3], elem_dofs [nelem, (p+1)^3], ndof, p as for Operator; ess [ndof]
    (nonzero = wall DoF); dt, nu; order 1..3; rtol of both solves; pressure_mode 0 (FP64
    PCG) or 1 (FP32 inner solves in FP64 refinement) with pressure_precond PRECOND_JACOBI;
    pressure_precond PRECOND_LOR32 (the default) preconditions the pressure Poisson solve
    by the LOR multigrid V-cycle (Section 5.2) in FP32 arithmetic inside FP64 CG,
    PRECOND_LOR by the same V-cycle in FP64.  velocity_mode 0 (FP64 PCG) or 1 (the default:
    FP32 inner solves in FP64 refinement) for the three-member Jacobi-preconditioned
    Helmholtz solve."""

    def __init__(self, elem_xyz, elem_dofs, ndof, p, ess, dt, nu, order=3, rtol=1e-10,
                 pressure_mode=1, device=None, check_every=8, maxit=10000, pressure_precond=None,
                 velocity_mode=1):
        check_mesh_shapes(np.shape(elem_xyz), np.shape(elem_dofs), ndof, p, np.shape(ess))
        if not 1 <= int(order) <= 3:
            raise ValueError("order 1, 2 or 3")
        self._lib = _lib.load()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the sfem library runs on MI355X (gfx950) only")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        dev = self.device
        self.ndof, self.p = int(ndof), int(p)
        self.dt, self.nu, self.order, self.rtol = float(dt), float(nu), int(order), float(rtol)
        self.pressure_mode = int(pressure_mode)
        xyz = torch.as_tensor(elem_xyz, dtype=torch.float64).to(dev).contiguous()
        dofs = torch.as_tensor(elem_dofs, dtype=torch.int32).to(dev).contiguous()
        essd = torch.as_tensor(np.asarray(ess)).to(dev).to(torch.uint8).contiguous()
        nelem = int(xyz.shape[0]) if xyz.ndim == 3 else 0
        self.pressure_precond = _lib.PRECOND_LOR32 if pressure_precond is None else int(pressure_precond)
        self.velocity_mode = int(velocity_mode)
        opts = FlowOpts(self.dt, self.nu, self.rtol, self.order, self.pressure_mode, int(check_every),
                        int(maxit), self.pressure_precond, self.velocity_mode)
        h = C.c_void_p()
        with torch.cuda.device(dev):
            st = self._lib.sfem_flow_create(dev.index, C.c_void_p(torch.cuda.current_stream(dev).cuda_stream),
                                            self.p, nelem, _ptr(xyz), _ptr(dofs), self.ndof, _ptr(essd),
                                            C.byref(opts), C.byref(h))
        if st != 0:
            raise SfemError(st, self._lib.sfem_flow_last_error(None).decode())
        self._h = h
        self.nstep = 0
        self.last = {}

    def close(self):
        if getattr(self, "_h", None):
            self._lib.sfem_flow_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _vec3(self, t, name):
        t = torch.as_tensor(t).to(device=self.device, dtype=torch.float64).contiguous()
        if tuple(t.shape) != (3, self.ndof):
            raise ValueError(f"{name} must have shape [3, ndof]")
        return t

    def step(self, u, f=None):
        """Advance from u = u^n [3, ndof] (float64, 0 on the walls); f = f^{n+1} [3, ndof]
        nodal or None.  Returns (u^{n+1}, p^{n+1}); per-solve outcomes in self.last."""
        u = self._vec3(u, "u")
        ff = None if f is None else self._vec3(f, "f")
        un = torch.empty_like(u)
        pn = torch.empty(self.ndof, dtype=torch.float64, device=self.device)
        self._lib.sfem_flow_set_stream(self._h, C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream))
        info = FlowInfo()
        st = self._lib.sfem_flow_step(self._h, _ptr(u), _ptr(ff), _ptr(un), _ptr(pn), C.byref(info))
        if st != 0:
            raise SfemError(st, f"projection step {self.nstep}: "
                                + self._lib.sfem_flow_last_error(self._h).decode())
        self.nstep += 1
        self.last = {"order": info.order,
                     "pressure": PcgResult([info.pressure], info.pressure.status),
                     "velocity": PcgResult(list(info.velocity),
                                           min((v.status for v in info.velocity), default=0))}
        return un, pn
