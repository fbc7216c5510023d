"""MI355X (gfx950) library for matrix-free, sum-factorized high-order hexahedral operators.

Python binding of the C ABI in ``include/sfem.h``: argument marshalling only.
Every step of the apply, diagonal, load, gradient and PCG runs in the HIP kernels
of ``libsfem.so``; PyTorch provides device memory and the stream.  If the library
is missing the import of this package still works, but creating an Operator raises
ImportError -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch  # loads the HIP runtime the library binds to

from . import _lib
from ._lib import (F32, F64, MASS, DIFFUSION, HELMHOLTZ, PRECOND_JACOBI, PRECOND_COLLOCATED_MASS,  # noqa: F401
                   PRECOND_LOR, PRECOND_LOR32, WEAK_GRADIENT, WEAK_CURL, WEAK_DIVERGENCE, SfemError, PcgOpts, PcgInfo,
                   CtxInfo, LorInfo)

__all__ = ["Operator", "SfemError", "MASS", "DIFFUSION", "HELMHOLTZ", "F64", "F32", "PcgResult",
           "WEAK_GRADIENT", "WEAK_CURL", "WEAK_DIVERGENCE", "ProjectionStepper"]


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else None


def check_mesh_shapes(xyz_shape, dofs_shape, ndof, p, ess_shape=None):
    """Raise ValueError unless the mesh arrays have the sizes sfem_setup reads:
    elem_xyz [nelem, 8, 3], elem_dofs [nelem, (p+1)^3] (or flat), ess [ndof]."""
    xyz_shape, dofs_shape = tuple(xyz_shape), tuple(dofs_shape)
    nelem = xyz_shape[0] if len(xyz_shape) == 3 else 0
    if len(xyz_shape) == 3 and xyz_shape[1:] != (8, 3):
        raise ValueError(f"elem_xyz must have shape [nelem, 8, 3], got {list(xyz_shape)}")
    if len(xyz_shape) != 3 and int(np.prod(xyz_shape)) != 0:
        raise ValueError(f"elem_xyz must have shape [nelem, 8, 3], got {list(xyz_shape)}")
    n3 = (int(p) + 1) ** 3
    if int(np.prod(dofs_shape)) != nelem * n3:
        raise ValueError(f"elem_dofs must hold nelem * (p+1)^3 = {nelem * n3} entries, "
                         f"got shape {list(dofs_shape)}")
    if ess_shape is not None and int(np.prod(tuple(ess_shape))) != int(ndof):
        raise ValueError(f"ess must hold ndof = {int(ndof)} entries, got shape {list(ess_shape)}")
    return nelem


def check_solve_shapes(b_shape, x_shape, ndof):
    """Raise ValueError unless b is [ndof] or [nbatch, ndof] and x (if given) has b's shape:
    sfem_pcg reads and writes nbatch * ndof values of both."""
    b_shape = tuple(b_shape)
    if len(b_shape) not in (1, 2) or b_shape[-1] != int(ndof):
        raise ValueError(f"b must have shape [ndof] or [nbatch, ndof] with ndof={int(ndof)}, "
                         f"got {list(b_shape)}")
    if x_shape is not None and tuple(x_shape) != b_shape:
        raise ValueError(f"x must have b's shape {list(b_shape)}, got {list(x_shape)}")


class PcgResult:
    """Per-member solver outcome (iterations, refinement steps, residuals, status)."""

    def __init__(self, infos, status):
        self.status = status
        self.iters = [i.iters for i in infos]
        self.outer = [i.outer for i in infos]
        self.rel_res = [i.rel_res for i in infos]
        self.true_rel_res = [i.true_rel_res for i in infos]
        self.member_status = [i.status for i in infos]

    @property
    def converged(self):
        return self.status == _lib.SFEM_OK

    def __repr__(self):
        return (f"PcgResult(status={_lib.STATUS_NAMES.get(self.status)}, iters={self.iters}, "
                f"outer={self.outer}, true_rel_res={self.true_rel_res})")


class Operator:
    """A set-up context: mesh + order p, quadrature data, coefficients.

    elem_xyz  [nelem, 8, 3] float64, elem_dofs [nelem, (p+1)^3] int32 (any array-likes;
    moved to the GPU), ndof, p, ess [ndof] (nonzero = essential) or None.
    """

    def __init__(self, elem_xyz, elem_dofs, ndof, p, ess=None, q=None, device=None):
        check_mesh_shapes(np.shape(elem_xyz), np.shape(elem_dofs), ndof, p,
                          None if ess is None else np.shape(ess))
        self._lib = _lib.load()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the sfem library runs on MI355X (gfx950) only")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.p = int(p)
        self.q = self.p + 2 if q is None else int(q)
        self.ndof = int(ndof)
        dev = self.device
        xyz = torch.as_tensor(elem_xyz, dtype=torch.float64).to(dev).contiguous()
        dofs = torch.as_tensor(elem_dofs, dtype=torch.int32).to(dev).contiguous()
        self.nelem = int(xyz.shape[0]) if xyz.ndim == 3 else 0
        essd = None
        if ess is not None:
            essd = torch.as_tensor(ess).to(dev).to(torch.uint8).contiguous()
        h = C.c_void_p()
        with torch.cuda.device(dev):
            st = self._lib.sfem_create(dev.index, C.c_void_p(torch.cuda.current_stream(dev).cuda_stream),
                                       C.byref(h))
        if st != 0:
            raise SfemError(st, self._lib.sfem_last_error(None).decode())
        self._h = h
        self._check(self._lib.sfem_setup(h, self.p, self.q, self.nelem, _ptr(xyz), _ptr(dofs),
                                         self.ndof, _ptr(essd)))
        self.nq = self.nelem * self.q ** 3
        self.nfields = 1

    # ---------------------------------------------------------------- plumbing
    def _check(self, st):
        if st < 0:
            raise SfemError(st, self._lib.sfem_last_error(self._h).decode())
        return st

    def _sync_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        self._lib.sfem_set_stream(self._h, C.c_void_p(s))

    def _vec(self, t, dtype, name):
        if not isinstance(t, torch.Tensor):
            t = torch.as_tensor(t)
        t = t.to(device=self.device, dtype=dtype).contiguous()
        if t.shape[-1] != self.ndof:
            raise ValueError(f"{name}: last dimension must be ndof={self.ndof}")
        return t

    def close(self):
        if getattr(self, "_h", None):
            self._lib.sfem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        ci = CtxInfo()
        self._check(self._lib.sfem_get_info(self._h, C.byref(ci)))
        return {k: getattr(ci, k) for k, _ in CtxInfo._fields_}

    # ---------------------------------------------------------------- operations
    def qpoint_coords(self):
        """Physical quadrature-point coordinates [3, nelem * q^3] (float64)."""
        self._sync_stream()
        out = torch.empty(3, self.nq, dtype=torch.float64, device=self.device)
        self._check(self._lib.sfem_qpoint_coords(self._h, _ptr(out)))
        return out

    def set_coeffs(self, alpha, beta, nu=None):
        """A = alpha M + beta K(nu); nu: [nelem, q^3], [nelem * q^3] or [nfield, nelem * q^3]."""
        self._sync_stream()
        nf = 1
        nud = None
        if nu is not None:
            nud = torch.as_tensor(nu).to(device=self.device, dtype=torch.float64).contiguous()
            if nud.numel() % self.nq != 0 or nud.numel() == 0:
                raise ValueError("nu must hold nelem * q^3 values per field")
            nf = nud.numel() // self.nq
        self._check(self._lib.sfem_set_coeffs(self._h, float(alpha), float(beta), _ptr(nud), nf))
        self.nfields = nf
        self.alpha, self.beta = float(alpha), float(beta)

    def apply(self, x, op=HELMHOLTZ, out=None):
        """y = A x; x float64 or float32, shape [ndof] or [nbatch, ndof]."""
        self._sync_stream()
        dtype = x.dtype if isinstance(x, torch.Tensor) and x.dtype in (torch.float32, torch.float64) \
            else torch.float64
        xv = self._vec(x, dtype, "x")
        if xv.ndim not in (1, 2):
            raise ValueError("x must have shape [ndof] or [nbatch, ndof]")
        nb = 1 if xv.ndim == 1 else xv.shape[0]
        y = torch.empty_like(xv) if out is None else out
        aliased = xv.numel() > 0 and y.data_ptr() == xv.data_ptr()
        if y.dtype != dtype or not y.is_contiguous() or y.shape != xv.shape or aliased:
            raise ValueError("out must be a distinct contiguous tensor of x's shape and dtype")
        prec = F32 if dtype == torch.float32 else F64
        self._check(self._lib.sfem_apply(self._h, op, prec, nb, _ptr(xv), _ptr(y)))
        return y

    def diagonal(self, op=HELMHOLTZ, dtype=torch.float64):
        """Exact diagonal of the constrained operator: [ndof] or [nfield, ndof]."""
        self._sync_stream()
        nf = 1 if op == MASS else self.nfields
        d = torch.empty(nf, self.ndof, dtype=dtype, device=self.device)
        prec = F32 if dtype == torch.float32 else F64
        self._check(self._lib.sfem_diagonal(self._h, op, prec, _ptr(d)))
        return d[0] if nf == 1 else d

    def load(self, f_q):
        """b = sum_q w|J| f_q phi (essential entries 0); f_q [nelem*q^3] or [nb, nelem*q^3]."""
        self._sync_stream()
        f = torch.as_tensor(f_q).to(device=self.device, dtype=torch.float64).contiguous()
        nb = 1 if f.numel() == self.nq else f.numel() // self.nq
        if f.numel() != nb * self.nq:
            raise ValueError("f_q must hold nelem * q^3 values per source")
        b = torch.empty(nb, self.ndof, dtype=torch.float64, device=self.device)
        self._check(self._lib.sfem_load(self._h, nb, _ptr(f), _ptr(b)))
        return b[0] if nb == 1 and f.ndim <= 1 else b

    def grad_nu(self, u, lam):
        """-beta (Gq grad lam).grad u per quadrature point: [nbatch, nelem * q^3] (or 1-D)."""
        self._sync_stream()
        uu = self._vec(u, torch.float64, "u")
        ll = self._vec(lam, torch.float64, "lam")
        if uu.shape != ll.shape:
            raise ValueError("u and lam must have the same shape")
        nb = 1 if uu.ndim == 1 else uu.shape[0]
        g = torch.empty(nb, self.nq, dtype=torch.float64, device=self.device)
        self._check(self._lib.sfem_grad_nu(self._h, nb, _ptr(uu), _ptr(ll), _ptr(g)))
        return g[0] if uu.ndim == 1 else g

    def setup_pressure(self, pres_dofs, npres):
        """Taylor-Hood pressure space (order p - 1) on the same elements: pres_dofs
        [nelem, p^3] int32 (local l = i + p (j + p k)), npres DoFs (no essential DoFs)."""
        self._sync_stream()
        d = torch.as_tensor(pres_dofs).to(device=self.device, dtype=torch.int32).contiguous()
        if d.numel() != self.nelem * self.p ** 3:
            raise ValueError("pres_dofs must hold nelem * p^3 entries")
        self._check(self._lib.sfem_setup_pressure(self._h, _ptr(d), int(npres)))
        self.npres = int(npres)

    def stokes_apply(self, u, pres):
        """Constrained Stokes block operator: (y_u [3, ndof], y_p [npres]) for u [3, ndof],
        pres [npres] (float64), with the Helmholtz coefficients of set_coeffs."""
        self._sync_stream()
        uu = self._vec(u, torch.float64, "u")
        if uu.ndim != 2 or uu.shape[0] != 3:
            raise ValueError("u must have shape [3, ndof]")
        pp = torch.as_tensor(pres).to(device=self.device, dtype=torch.float64).contiguous()
        if pp.numel() != getattr(self, "npres", -1):
            raise ValueError("pres must hold npres values (call setup_pressure first)")
        yu = torch.empty_like(uu)
        yp = torch.empty_like(pp)
        self._check(self._lib.sfem_stokes_apply(self._h, _ptr(uu), _ptr(pp), _ptr(yu), _ptr(yp)))
        return yu, yp

    def convection(self, u):
        """Convection term N(u) [3, ndof] (float64) for the velocity u [3, ndof]; rows of
        essential DoFs are 0."""
        self._sync_stream()
        uu = self._vec(u, torch.float64, "u")
        if uu.ndim != 2 or uu.shape[0] != 3:
            raise ValueError("u must have shape [3, ndof]")
        y = torch.empty_like(uu)
        self._check(self._lib.sfem_convection(self._h, _ptr(uu), _ptr(y)))
        return y

    def weak_op(self, kind, x):
        """Equal-order weak gradient ([ndof] -> [3, ndof]), curl ([3, ndof] -> [3, ndof]) or
        divergence ([3, ndof] -> [ndof]) of the projection step (float64); rows of
        essential DoFs are 0."""
        self._sync_stream()
        xx = self._vec(x, torch.float64, "x")
        nin = 1 if kind == WEAK_GRADIENT else 3
        if (nin == 1 and xx.ndim != 1) or (nin == 3 and (xx.ndim != 2 or xx.shape[0] != 3)):
            raise ValueError("x must have shape [ndof] (gradient) or [3, ndof] (curl, divergence)")
        shape = (self.ndof,) if kind == WEAK_DIVERGENCE else (3, self.ndof)
        y = torch.empty(shape, dtype=torch.float64, device=self.device)
        self._check(self._lib.sfem_weak_op(self._h, int(kind), _ptr(xx), _ptr(y)))
        return y

    def lincomb(self, coefs, xs, scale=None, mask=None, out=None):
        """sum_j coefs[j] xs[j], divided by scale [ndof] and zeroed where mask [ndof] != 0
        (both optional); every xs[j] of the same shape [..., ndof] (float64)."""
        self._sync_stream()
        xs = [self._vec(x, torch.float64, "x") for x in xs]
        if len(xs) != len(coefs) or not xs or any(x.shape != xs[0].shape for x in xs):
            raise ValueError("one coefficient per input, all inputs of one shape")
        nb = xs[0].numel() // self.ndof
        sc = None if scale is None else self._vec(scale, torch.float64, "scale")
        mk = None if mask is None else self._vec(mask, torch.uint8, "mask")
        y = torch.empty_like(xs[0]) if out is None else out
        if y.shape != xs[0].shape or y.dtype != torch.float64 or not y.is_contiguous():
            raise ValueError("out must be a contiguous float64 tensor of the inputs' shape")
        cf = (C.c_double * len(xs))(*[float(c) for c in coefs])
        pv = (C.c_void_p * len(xs))(*[x.data_ptr() for x in xs])
        self._check(self._lib.sfem_lincomb(self._h, len(xs), cf, pv, _ptr(sc), _ptr(mk), self.ndof,
                                           nb, _ptr(y)))
        return y

    def collocated_mass(self):
        """Collocated (GLL-integrated) mass diagonal [ndof], essential entries 1 (float64)."""
        self._sync_stream()
        d = torch.empty(self.ndof, dtype=torch.float64, device=self.device)
        self._check(self._lib.sfem_collocated_mass(self._h, _ptr(d)))
        return d

    def lor_setup(self, op=HELMHOLTZ):
        """Build the LOR multigrid of operator kind op (Section 5.2); returns its level sizes
        and nonzeros, the host setup time and the device storage per level ("sliced": bit 0
        the operator, bit 1 the prolongator, bit 2 the restriction in sliced ELL, bit 3
        operator slices with a shared column-offset pattern)."""
        self._sync_stream()
        info = LorInfo()
        self._check(self._lib.sfem_lor_setup(self._h, op, C.byref(info)))
        L = info.levels
        return {"levels": L, "rows": list(info.rows[:L]), "nnz": list(info.nnz[:L]),
                "setup_ms": info.setup_ms, "sliced": list(info.sliced[:L])}

    def lor_apply(self, x, op=HELMHOLTZ):
        """y = A_LOR x (float64 [ndof])."""
        self._sync_stream()
        xv = self._vec(x, torch.float64, "x")
        if xv.ndim != 1:
            raise ValueError("x must have shape [ndof]")
        y = torch.empty_like(xv)
        self._check(self._lib.sfem_lor_apply(self._h, op, _ptr(xv), _ptr(y)))
        return y

    def lor_vcycle(self, b, op=HELMHOLTZ, prec=F64):
        """One multigrid V-cycle for A_LOR x = b from x = 0 (float64 [ndof] in and out);
        prec=F32 runs it with FP32 copies of the hierarchy and FP32 vectors."""
        self._sync_stream()
        bv = self._vec(b, torch.float64, "b")
        if bv.ndim != 1:
            raise ValueError("b must have shape [ndof]")
        x = torch.empty_like(bv)
        self._check(self._lib.sfem_lor_vcycle(self._h, op, int(prec), _ptr(bv), _ptr(x)))
        return x

    def pcg(self, b, x=None, op=HELMHOLTZ, rtol=1e-10, maxit=10000, mode=0, inner_rtol=1e-5,
            max_outer=30, check_every=8, precond=PRECOND_JACOBI, nullspace=False):
        """Preconditioned CG (mode 0) or FP32-inner CG inside FP64 refinement (mode 1).
        precond: PRECOND_JACOBI (exact operator diagonal), PRECOND_COLLOCATED_MASS, or
        PRECOND_LOR (a multigrid V-cycle on the low-order-refined operator; mode 0), or
        PRECOND_LOR32 (that V-cycle in FP32 arithmetic inside FP64 CG; mode 0).
        nullspace=True: pure-Neumann diffusion solve (no
        essential DoFs) with the preconditioner orthogonalized against the constants and
        the mean-zero solution returned.

        Returns (x, PcgResult).  Raises SfemError on errors; a non-converged solve
        returns the last iterate with status SFEM_NOCONV.
        """
        self._sync_stream()
        bv = self._vec(b, torch.float64, "b")
        check_solve_shapes(bv.shape, None if x is None else np.shape(x), self.ndof)
        nb = 1 if bv.ndim == 1 else bv.shape[0]
        x0_zero = x is None
        xv = torch.empty_like(bv) if x0_zero else self._vec(x, torch.float64, "x").clone()
        opts = PcgOpts(float(rtol), int(maxit), int(mode), float(inner_rtol), int(max_outer),
                       int(check_every), 1 if x0_zero else 0, int(precond), 1 if nullspace else 0)
        infos = (PcgInfo * nb)()
        st = self._check(self._lib.sfem_pcg(self._h, op, nb, _ptr(bv), _ptr(xv), C.byref(opts), infos))
        return xv, PcgResult(list(infos), st)


from .flow import ProjectionStepper  # noqa: E402,F401
