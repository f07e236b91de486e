"""Python binding of the boundary-element entry points (bem_setup,
bem_matvec, bem_rhs, bem_energy, bem_precondition, gmres_solve).

The mesh is passed as host arrays; vectors are float64 CUDA tensors of
length 2 * n_unknowns ([u; v]): n_triangles for P0 elements, n_vertices for
P1.  Every step runs in libfmmbem.so."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import check, lib
from .fmm import PRECISIONS, _ptr, _stream

FORMULATIONS = {"direct": _lib.FMM_BEM_DIRECT, "derivative": _lib.FMM_BEM_DERIVATIVE,
                "exterior": _lib.FMM_BEM_EXTERIOR, "exterior_p1": _lib.FMM_BEM_EXTERIOR_P1}
PRECONDITIONERS = {"block": _lib.FMM_BEM_PRECOND_BLOCK, "mass": _lib.FMM_BEM_PRECOND_MASS}


class BEMOperator:
    """P0 boundary-element operator on a triangle mesh (regular rule with
    quad_pts points): formulation "direct", [[M/2 + K_L, -V_L], [M/2 - K_Y,
    (eps_in/eps_out) V_Y]], "derivative" (Juffer), [[(1+e21)/2 M - (e21 K_Y -
    K_L), V_Y - V_L], [W_Y - W_L, (1+e12)/2 M + e12 K'_Y - K'_L]], or "exterior"
    (Lu), [[(1+e12)/2 M - (K_Y - e12 K_L), V_Y - V_L], [e12 (W_Y - W_L), (1+e12)/2
    M + e12 K'_Y - K'_L]] for the solvent-side unknowns; "exterior_p1": the
    same on continuous piecewise-linear elements (unknowns per vertex, P1 mass
    matrix).  preconditioner: "block" (per-triangle 2 x 2 block-diagonal, P0
    only) or "mass" (diag(M, M), lumped for P1); None: "mass" for P1, "block"
    otherwise."""

    def __init__(self, verts, tris, quad_pts: int = 3, eps_in: float = 4.0, eps_out: float = 80.0,
                 kappa: float = 0.125, p: int = 6, ncrit: int = 128, precision: str = "fp32", device="cuda",
                 formulation: str = "direct", preconditioner: str | None = None):
        v = np.ascontiguousarray(verts, dtype=np.float64)
        t = np.ascontiguousarray(tris, dtype=np.int32)
        if v.ndim != 2 or v.shape[1] != 3 or t.ndim != 2 or t.shape[1] != 3:
            raise ValueError("verts (nv,3) and tris (nt,3) expected")
        self.nt = int(t.shape[0])
        self.device = torch.device(device)
        self.precision = precision
        if formulation not in FORMULATIONS:
            raise ValueError(f"unknown formulation {formulation!r}")
        self.formulation = formulation
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(lib().bem_setup(ctypes.c_void_p(v.ctypes.data), v.shape[0], ctypes.c_void_p(t.ctypes.data), self.nt,
                                  int(quad_pts), float(eps_in), float(eps_out), float(kappa), int(p), int(ncrit),
                                  PRECISIONS[precision], FORMULATIONS[formulation], _stream(), ctypes.byref(h)),
                  "bem_setup")
        self._h = h
        self.nu = self.info()["n_unknowns"]
        if preconditioner is None:
            preconditioner = "mass" if formulation == "exterior_p1" else "block"
        self.set_preconditioner(preconditioner)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().bem_free(h)
            except Exception:
                pass
            self._h = None

    def _vec(self, x):
        x = x.to(device=self.device, dtype=torch.float64).contiguous()
        if x.shape != (2 * self.nu,):
            raise ValueError(f"expected a vector of length {2 * self.nu}")
        return x

    def matvec(self, x):
        x = self._vec(x)
        y = torch.empty_like(x)
        check(lib().bem_matvec(self._h, _ptr(x), _ptr(y), _stream()), "bem_matvec")
        return y

    def set_preconditioner(self, kind: str):
        if kind not in PRECONDITIONERS:
            raise ValueError(f"unknown preconditioner {kind!r}")
        check(lib().bem_set_preconditioner(self._h, PRECONDITIONERS[kind], _stream()), "bem_set_preconditioner")
        self.preconditioner = kind

    def precondition(self, x):
        x = self._vec(x)
        y = torch.empty_like(x)
        check(lib().bem_precondition(self._h, _ptr(x), _ptr(y), _stream()), "bem_precondition")
        return y

    def rhs(self, qxyz, q):
        qx = torch.as_tensor(qxyz, dtype=torch.float64).to(self.device).contiguous().reshape(-1, 3)
        qq = torch.as_tensor(q, dtype=torch.float64).to(self.device).contiguous().reshape(-1)
        b = torch.empty(2 * self.nu, dtype=torch.float64, device=self.device)
        check(lib().bem_rhs(self._h, _ptr(qx), _ptr(qq), qq.numel(), _ptr(b), _stream()), "bem_rhs")
        return b

    def energy(self, x, qxyz, q) -> float:
        x = self._vec(x)
        qx = torch.as_tensor(qxyz, dtype=torch.float64).to(self.device).contiguous().reshape(-1, 3)
        qq = torch.as_tensor(q, dtype=torch.float64).to(self.device).contiguous().reshape(-1)
        out = ctypes.c_double()
        check(lib().bem_energy(self._h, _ptr(x), _ptr(qx), _ptr(qq), qq.numel(), ctypes.byref(out), _stream()),
              "bem_energy")
        return out.value

    def solve(self, b, x0=None, tol: float = 1e-6, maxiter: int = 500, restart: int = 0,
              refine: "BEMOperator | None" = None, inner_tol: float = 1e-4):
        """gmres(self, b, ...): (x, iterations, residual history, status)."""
        return gmres(self, b, x0=x0, tol=tol, maxiter=maxiter, restart=restart, refine=refine, inner_tol=inner_tol)

    def info(self) -> dict:
        raw = ctypes.create_string_buffer(48)
        check(lib().bem_info(self._h, raw), "bem_info")
        a = np.frombuffer(raw.raw[:24], dtype=np.int64)
        b = np.frombuffer(raw.raw[24:40], dtype=np.int32)
        c = np.frombuffer(raw.raw[40:48], dtype=np.int64)
        return {"n_triangles": int(a[0]), "n_points": int(a[1]), "n_singular_pairs": int(a[2]),
                "quad_pts": int(b[0]), "precision": int(b[1]), "formulation": int(b[2]),
                "preconditioner": int(b[3]), "n_unknowns": int(c[0])}


def gmres(op: BEMOperator, b, x0=None, tol: float = 1e-6, maxiter: int = 500, restart: int = 0,
          refine: BEMOperator | None = None, inner_tol: float = 1e-4):
    """FP64 right-preconditioned GMRES (optionally with iterative refinement
    against `refine`).  Returns (x, iterations, residual history, status)."""
    b = op._vec(b)
    x = torch.zeros_like(b) if x0 is None else op._vec(x0).clone()
    it = ctypes.c_int()
    hist = np.zeros(maxiter)
    rc = lib().gmres_solve(op._h, refine._h if refine is not None else None, _ptr(b), _ptr(x), float(tol),
                           float(inner_tol), int(maxiter), int(restart), ctypes.byref(it),
                           ctypes.c_void_p(hist.ctypes.data), _stream())
    if rc not in (_lib.FMM_OK, _lib.FMM_ENOTCONV):
        check(rc, "gmres_solve")
    return x, it.value, hist[:it.value].copy(), rc
