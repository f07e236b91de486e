"""Python binding of the FMM entry points (fmm_setup / fmm_eval / fmm_free).

Torch tensors supply device memory and the current HIP stream; every step of
the evaluation runs in libfmmbem.so."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import check, lib

KERNELS = {"laplace": _lib.FMM_LAPLACE, "yukawa": _lib.FMM_YUKAWA}
PRECISIONS = {"fp64": _lib.FMM_FP64, "fp32": _lib.FMM_FP32, "bf16x3": _lib.FMM_FP32_BF16X3}


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class FMMPlan:
    """A kernel-independent FMM plan for a fixed point set (targets = sources),
    or, with `offsets`, for a batch of independent point sets (molecule m is
    points offsets[m]:offsets[m+1]; molecules do not interact).

    points: (N, 3) float64 CUDA tensor (copied and sorted by the library).
    kernel: "laplace" or "yukawa"; kappa >= 0; p: points per surface edge;
    ncrit: maximum points per leaf; precision: "fp64", "fp32" or "bf16x3"."""

    def __init__(self, points: torch.Tensor, kernel: str = "laplace", kappa: float = 0.0, p: int = 6,
                 ncrit: int = 64, precision: str = "fp32", offsets=None):
        if kernel not in KERNELS:
            raise ValueError(f"unknown kernel {kernel!r}")
        if precision not in PRECISIONS:
            raise ValueError(f"unknown precision {precision!r}")
        pts = points.detach().to(dtype=torch.float64).contiguous()
        if pts.ndim != 2 or pts.shape[1] != 3 or not pts.is_cuda:
            raise ValueError("points must be an (N, 3) CUDA tensor")
        self.n = int(pts.shape[0])
        self.kernel, self.kappa, self.p, self.ncrit, self.precision = kernel, float(kappa), int(p), int(ncrit), precision
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        self.device = pts.device
        h = ctypes.c_void_p()
        with torch.cuda.device(pts.device):
            if offsets is None:
                check(lib().fmm_setup(_ptr(pts), self.n, KERNELS[kernel], self.kappa, self.p, self.ncrit,
                                      PRECISIONS[precision], _stream(), ctypes.byref(h)), "fmm_setup")
            else:
                off = np.ascontiguousarray(offsets, dtype=np.int64)
                if off.ndim != 1 or off[0] != 0 or off[-1] != self.n:
                    raise ValueError("offsets must start at 0 and end at the number of points")
                check(lib().fmm_setup_batch(_ptr(pts), ctypes.c_void_p(off.ctypes.data), len(off) - 1,
                                            KERNELS[kernel], self.kappa, self.p, self.ncrit, PRECISIONS[precision],
                                            _stream(), ctypes.byref(h)), "fmm_setup_batch")
        self._h = h
        # the FP64 points the tree was built from (the caller's tensor itself
        # when it already was contiguous FP64), for check_points
        self._points = pts
        self._points_version = pts._version

    def check_points(self, xyz: torch.Tensor):
        """Raise ValueError unless xyz holds exactly the points this plan was
        built from (same shape and device, equal values, not modified in place
        since the setup)."""
        if self._points._version != self._points_version:
            raise ValueError("the plan's points were modified in place after the plan was built")
        if tuple(xyz.shape) != (self.n, 3) or xyz.device != self.device:
            raise ValueError(f"xyz must be an ({self.n}, 3) tensor on {self.device}, the plan's points")
        if (xyz.dtype == torch.float64 and xyz.is_contiguous() and xyz.data_ptr() == self._points.data_ptr()):
            return
        if not torch.equal(xyz.detach().to(torch.float64), self._points):
            raise ValueError("xyz differs from the points the plan was built from; build a new plan")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().fmm_free(h)
            except Exception:
                pass
            self._h = None

    def eval(self, q: torch.Tensor, gradient: bool = True, out=None):
        """q: (N,) or (nrhs, N) densities.  Returns (pot, grad) with shapes
        (nrhs, N) and (nrhs, N, 3) (leading dim dropped for 1-D q)."""
        squeeze = q.ndim == 1
        qq = q.reshape(1, -1) if squeeze else q
        if qq.shape[1] != self.n:
            raise ValueError("density length does not match the plan")
        qq = qq.to(device=self.device, dtype=self.dtype).contiguous()
        nrhs = int(qq.shape[0])
        if out is None:
            pot = torch.empty((nrhs, self.n), dtype=self.dtype, device=self.device)
            grad = torch.empty((nrhs, self.n, 3), dtype=self.dtype, device=self.device) if gradient else None
        else:
            pot, grad = out
        check(lib().fmm_eval(self._h, _ptr(qq), nrhs, _ptr(pot), _ptr(grad), _stream()), "fmm_eval")
        if squeeze:
            return pot[0], (grad[0] if grad is not None else None)
        return pot, grad

    __call__ = eval

    def set_profiling(self, enable=True, serial=False):
        """enable: True (every phase), False, or an iterable of phase names.
        serial: pair evaluations led by this plan run every pass on the
        caller's stream one after the other (phase times not stretched by
        overlap; for measurement)."""
        if enable is True:
            mask = (1 << len(_lib.PHASES)) - 1
        elif not enable:
            mask = 0
        else:
            mask = 0
            for name in enable:
                mask |= 1 << _lib.PHASES.index(name)
        if serial:
            mask |= _lib.FMM_PROFILE_SERIAL
        check(lib().fmm_set_profiling(self._h, mask), "fmm_set_profiling")

    def phase_times(self) -> dict:
        """Accumulated per-phase milliseconds and launch counts since the last
        call (synchronises on the recorded events)."""
        n = len(_lib.PHASES)
        ms = np.zeros(n)
        cnt = np.zeros(n, np.int64)
        check(lib().fmm_get_phase_times(self._h, ctypes.c_void_p(ms.ctypes.data), ctypes.c_void_p(cnt.ctypes.data), n),
              "fmm_get_phase_times")
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(_lib.PHASES)}

    def info(self) -> dict:
        inf = _lib.FmmInfo()
        check(lib().fmm_info(self._h, ctypes.byref(inf)), "fmm_info")
        return {k: getattr(inf, k) for k, _ in _lib.FmmInfo._fields_}

    def tree(self) -> dict:
        inf = self.info()
        n, nb = inf["n_points"], inf["n_boxes"]
        nl = inf["n_u_pairs"] + inf["n_v_pairs"] + inf["n_w_pairs"] + inf["n_x_pairs"]
        a = {
            "perm": np.zeros(n, np.int64), "keys": np.zeros(n, np.int64), "level": np.zeros(nb, np.int32),
            "anchor": np.zeros((nb, 3), np.int64), "begin": np.zeros(nb, np.int64), "end": np.zeros(nb, np.int64),
            "parent": np.zeros(nb, np.int64), "child_begin": np.zeros(nb, np.int64), "nchild": np.zeros(nb, np.int32),
            "list_off": np.zeros(4 * (nb + 1), np.int64), "list_idx": np.zeros(max(nl, 1), np.int64),
        }
        order = ["perm", "keys", "level", "anchor", "begin", "end", "parent", "child_begin", "nchild", "list_off",
                 "list_idx"]
        check(lib().fmm_get_tree(self._h, *[ctypes.c_void_p(a[k].ctypes.data) for k in order]), "fmm_get_tree")
        off = a["list_off"].reshape(4, nb + 1)
        lists = []
        for k in range(4):
            lists.append([a["list_idx"][off[k, b]:off[k, b + 1]].tolist() for b in range(nb)])
        a["U"], a["V"], a["W"], a["X"] = lists
        lo = np.zeros(3)
        w = ctypes.c_double()
        check(lib().fmm_get_root(self._h, ctypes.c_void_p(lo.ctypes.data), ctypes.byref(w)), "fmm_get_root")
        a["lo"], a["W_root"] = lo, w.value
        return a


def eval_pair(plan_a: FMMPlan, plan_b: FMMPlan, q: torch.Tensor, gradient: bool = True):
    """Both plans on the same densities (fmm_eval_pair): returns
    ((pot_a, grad_a), (pot_b, grad_b)) with the shapes of FMMPlan.eval.  A
    Laplace plan_a and a Yukawa plan_b on the same points, p, ncrit and
    precision share one tree and one near-field launch."""
    if plan_a.n != plan_b.n or plan_a.dtype != plan_b.dtype:
        raise ValueError("plans differ in point count or precision")
    squeeze = q.ndim == 1
    qq = q.reshape(1, -1) if squeeze else q
    if qq.shape[1] != plan_a.n:
        raise ValueError("density length does not match the plans")
    qq = qq.to(device=plan_a.device, dtype=plan_a.dtype).contiguous()
    nrhs = int(qq.shape[0])
    outs = []
    for _ in range(2):
        pot = torch.empty((nrhs, plan_a.n), dtype=plan_a.dtype, device=plan_a.device)
        grad = torch.empty((nrhs, plan_a.n, 3), dtype=plan_a.dtype, device=plan_a.device) if gradient else None
        outs.append((pot, grad))
    (pa, ga), (pb, gb) = outs
    check(lib().fmm_eval_pair(plan_a._h, plan_b._h, _ptr(qq), nrhs, _ptr(pa), _ptr(ga), _ptr(pb), _ptr(gb),
                              _stream()), "fmm_eval_pair")
    if squeeze:
        return (pa[0], ga[0] if ga is not None else None), (pb[0], gb[0] if gb is not None else None)
    return (pa, ga), (pb, gb)


def eval_pair_md(plan_a: FMMPlan, plan_b: FMMPlan, q: torch.Tensor, dip: torch.Tensor, qscale_a: float = 1.0,
                 qscale_b: float = 1.0, gradient: bool = False):
    """Potentials of monopole (q, (N,)) and dipole (dip, (N, 3)) sources for a
    Laplace plan_a and a Yukawa plan_b sharing one tree (fmm_eval_pair_md):
    pot_k = qscale_k G_k q + sum_j dip_j . grad_y g_k.  Returns (pot_a, pot_b),
    or ((pot_a, grad_a), (pot_b, grad_b)) with gradient=True."""
    n = plan_a.n
    qq = q.reshape(-1).to(device=plan_a.device, dtype=plan_a.dtype).contiguous()
    dd = dip.reshape(-1, 3).to(device=plan_a.device, dtype=plan_a.dtype).contiguous()
    if qq.numel() != n or dd.shape[0] != n:
        raise ValueError("q and dip must have one entry per point")
    pa = torch.empty(n, dtype=plan_a.dtype, device=plan_a.device)
    pb = torch.empty(n, dtype=plan_a.dtype, device=plan_a.device)
    ga = torch.empty((n, 3), dtype=plan_a.dtype, device=plan_a.device) if gradient else None
    gb = torch.empty((n, 3), dtype=plan_a.dtype, device=plan_a.device) if gradient else None
    check(lib().fmm_eval_pair_md(plan_a._h, plan_b._h, _ptr(qq), _ptr(dd), float(qscale_a), float(qscale_b),
                                 _ptr(pa), _ptr(ga), _ptr(pb), _ptr(gb), _stream()), "fmm_eval_pair_md")
    if gradient:
        return (pa, ga), (pb, gb)
    return pa, pb
