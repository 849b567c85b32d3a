"""Python binding of fqp_solve_batch: torch device tensors in, torch device
tensors out.  Every step of the solve runs in libfqp's HIP kernels; this
module only lays out arrays and marshals pointers.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from . import _lib


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def pack_eligibility(elig: np.ndarray) -> np.ndarray:
    """bool [m, n] -> uint32 [m, ceil(n/32)], bit i%32 of word i//32."""
    m, n = elig.shape
    W = (n + 31) // 32
    by = np.packbits(elig.astype(np.uint8), axis=1, bitorder="little")
    pad = np.zeros((m, 4 * W), dtype=np.uint8)
    pad[:, :by.shape[1]] = by
    return pad.view("<u4").reshape(m, W).copy()


@dataclass
class DeviceProblem:
    """Universe + book laid out on the device as the C-ABI expects."""
    n: int
    k: int
    G: int
    m: int
    B: torch.Tensor
    f: torch.Tensor
    d: torch.Tensor
    group: Optional[torch.Tensor]
    mu: torch.Tensor
    w0: torch.Tensor
    lb: torch.Tensor
    ub: torch.Tensor
    eligible: Optional[torch.Tensor]
    gamma: torch.Tensor
    kappa: torch.Tensor
    tau: torch.Tensor
    band_lo: Optional[torch.Tensor]
    band_hi: Optional[torch.Tensor]
    tax_ptr: Optional[torch.Tensor]
    tax_asset: Optional[torch.Tensor]
    tax_brk: Optional[torch.Tensor]
    tax_slope: Optional[torch.Tensor]
    # the rest of Eq. 1 (optional): halfspace rows [H, n] shared by the book
    # with per-account bounds [m, H]; per-asset bounds [m, n]; benchmark
    # weights [m, n] and return scale [m]
    H: int = 0
    half: Optional[torch.Tensor] = None
    half_lo: Optional[torch.Tensor] = None
    half_hi: Optional[torch.Tensor] = None
    lb_asset: Optional[torch.Tensor] = None
    ub_asset: Optional[torch.Tensor] = None
    wb: Optional[torch.Tensor] = None
    eta: Optional[torch.Tensor] = None

    @property
    def n_rows(self) -> int:
        """constraint rows: bands, then halfspaces"""
        return self.G + self.H


def subset(P: DeviceProblem, idx) -> DeviceProblem:
    """The accounts ``idx`` of a device book (same universe, same device)."""
    idx_l = [int(a) for a in idx]
    it = torch.as_tensor(idx_l, dtype=torch.long, device=P.mu.device)
    rows = (lambda t: None if t is None else t.index_select(0, it).contiguous())
    tax_ptr = tax_asset = tax_brk = tax_slope = None
    if P.tax_ptr is not None:
        ptr = P.tax_ptr.cpu().numpy()
        sel = np.concatenate([np.arange(ptr[a], ptr[a + 1]) for a in idx_l]).astype(np.int64) \
            if idx_l else np.zeros(0, np.int64)
        new_ptr = np.concatenate([[0], np.cumsum([ptr[a + 1] - ptr[a] for a in idx_l])])
        st = torch.as_tensor(sel, device=P.mu.device)
        tax_ptr = torch.as_tensor(new_ptr.astype(np.int32), device=P.mu.device)
        tax_asset = P.tax_asset.index_select(0, st).contiguous()
        tax_brk = P.tax_brk.index_select(0, st).contiguous()
        tax_slope = P.tax_slope.index_select(0, st).contiguous()
    return DeviceProblem(
        n=P.n, k=P.k, G=P.G, m=len(idx_l), B=P.B, f=P.f, d=P.d, group=P.group,
        mu=rows(P.mu), w0=rows(P.w0), lb=rows(P.lb), ub=rows(P.ub),
        eligible=rows(P.eligible), gamma=rows(P.gamma), kappa=rows(P.kappa),
        tau=rows(P.tau), band_lo=rows(P.band_lo), band_hi=rows(P.band_hi),
        tax_ptr=tax_ptr, tax_asset=tax_asset, tax_brk=tax_brk, tax_slope=tax_slope,
        H=P.H, half=P.half, half_lo=rows(P.half_lo), half_hi=rows(P.half_hi),
        lb_asset=rows(P.lb_asset), ub_asset=rows(P.ub_asset), wb=rows(P.wb), eta=rows(P.eta))


def to_device(uni, book, device="cuda:0") -> DeviceProblem:
    """Lay out a (workloads.Universe, workloads.Book) pair on the device."""
    dev = torch.device(device)

    def f32(x):
        return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float32),
                               device=dev)

    def i32(x):
        return torch.as_tensor(np.ascontiguousarray(x, dtype=np.int32),
                               device=dev)

    G = uni.n_groups if book.band_lo is not None else 0
    H = getattr(uni, "n_half", 0) if getattr(book, "half_lo", None) is not None else 0
    opt = (lambda x: None if x is None else f32(x))
    elig = None
    if not book.eligible.all():
        elig = torch.as_tensor(pack_eligibility(book.eligible).view(np.int32),
                               device=dev)
    has_tax = book.tax_asset.size > 0
    return DeviceProblem(
        n=uni.n, k=uni.k, G=G, m=book.m,
        B=f32(uni.B), f=f32(uni.f), d=f32(uni.d),
        group=i32(uni.group) if G else None,
        mu=f32(book.mu), w0=f32(book.w0), lb=f32(book.lb), ub=f32(book.ub),
        eligible=elig, gamma=f32(book.gamma), kappa=f32(book.kappa),
        tau=f32(book.tau),
        band_lo=f32(book.band_lo) if G else None,
        band_hi=f32(book.band_hi) if G else None,
        tax_ptr=i32(book.tax_ptr) if has_tax else None,
        tax_asset=i32(book.tax_asset) if has_tax else None,
        tax_brk=f32(book.tax_brk) if has_tax else None,
        tax_slope=f32(book.tax_slope) if has_tax else None,
        H=H, half=f32(uni.half) if H else None,
        half_lo=f32(book.half_lo) if H else None, half_hi=f32(book.half_hi) if H else None,
        lb_asset=opt(getattr(book, "lb_asset", None)), ub_asset=opt(getattr(book, "ub_asset", None)),
        wb=opt(getattr(book, "wb", None)), eta=opt(getattr(book, "eta", None)),
    )


SETTING_NAMES = [name for name, _ in _lib.Settings._fields_]


class Solver:
    """Owns one library handle (and its device workspace)."""

    def __init__(self, device: int = 0):
        self.lib = _lib.load()
        self.device = device
        h = ctypes.c_void_p()
        rc = self.lib.fqp_create(ctypes.byref(h), device)
        if rc != 0:
            raise RuntimeError(
                f"fqp_create failed: {self.lib.fqp_error_string(rc).decode()}")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.fqp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def settings(self, **kw) -> _lib.Settings:
        s = _lib.Settings()
        self.lib.fqp_default_settings(ctypes.byref(s))
        for key, val in kw.items():
            if key not in SETTING_NAMES:
                raise KeyError(f"unknown setting {key!r}")
            setattr(s, key, val)
        return s

    def solve(self, P: DeviceProblem, out: Optional[dict] = None, stream=None,
              warm_state: Optional[torch.Tensor] = None, want_state: bool = False,
              **settings) -> dict:
        """Solve every account of P.  ``warm_state`` (float32, the ``state``
        output of an earlier solve of the same accounts, from any Solver)
        seeds a warm start when settings carry warm_start=1; ``want_state``
        adds that output ("state") for a later warm start."""
        dev = P.mu.device
        m, n, G = P.m, P.n, P.n_rows
        nstate = _lib.state_floats(m, n, G)
        if warm_state is not None:
            if warm_state.dtype != torch.float32 or warm_state.numel() != nstate \
                    or not warm_state.is_contiguous() or warm_state.device != dev:
                raise ValueError(f"warm_state: {nstate} contiguous float32 values on {dev}")
        if out is None:
            out = dict(
                w=torch.empty((m, n), dtype=torch.float64, device=dev),
                status=torch.empty(m, dtype=torch.int32, device=dev),
                iters=torch.empty(m, dtype=torch.int32, device=dev),
                r_prim=torch.empty(m, dtype=torch.float64, device=dev),
                r_dual=torch.empty(m, dtype=torch.float64, device=dev),
                r_comp=torch.empty(m, dtype=torch.float64, device=dev),
                obj=torch.empty(m, dtype=torch.float64, device=dev),
                nu=torch.empty(m, dtype=torch.float64, device=dev),
                lam_cap=torch.empty(m, dtype=torch.float64, device=dev),
                lam_band=torch.zeros((m, max(G, 1)), dtype=torch.float64,
                                     device=dev),
            )
        if want_state and "state" not in out:
            out["state"] = torch.empty(nstate, dtype=torch.float32, device=dev)
        U = _lib.Universe(n=n, k=P.k, n_groups=P.G, B=_ptr(P.B), f=_ptr(P.f),
                          d=_ptr(P.d), group=_ptr(P.group), n_half=P.H, half=_ptr(P.half))
        Bk = _lib.Book(m=m, mu=_ptr(P.mu), w0=_ptr(P.w0), lb=_ptr(P.lb),
                       ub=_ptr(P.ub), eligible=_ptr(P.eligible),
                       gamma=_ptr(P.gamma), kappa=_ptr(P.kappa),
                       tau=_ptr(P.tau), band_lo=_ptr(P.band_lo),
                       band_hi=_ptr(P.band_hi), tax_ptr=_ptr(P.tax_ptr),
                       tax_asset=_ptr(P.tax_asset), tax_brk=_ptr(P.tax_brk),
                       tax_slope=_ptr(P.tax_slope), warm_state=_ptr(warm_state),
                       lb_asset=_ptr(P.lb_asset), ub_asset=_ptr(P.ub_asset),
                       half_lo=_ptr(P.half_lo), half_hi=_ptr(P.half_hi),
                       wb=_ptr(P.wb), eta=_ptr(P.eta))
        R = _lib.Result(w=_ptr(out["w"]), status=_ptr(out["status"]),
                        iters=_ptr(out["iters"]), r_prim=_ptr(out["r_prim"]),
                        r_dual=_ptr(out["r_dual"]),
                        r_comp=_ptr(out["r_comp"]), obj=_ptr(out["obj"]),
                        nu=_ptr(out["nu"]), lam_cap=_ptr(out["lam_cap"]),
                        lam_band=_ptr(out["lam_band"]) if G else None,
                        state=_ptr(out.get("state")))
        S = self.settings(**settings)
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        rc = self.lib.fqp_solve_batch(self.h, ctypes.byref(U), ctypes.byref(Bk),
                                      ctypes.byref(S), ctypes.byref(R),
                                      ctypes.c_void_p(stream.cuda_stream))
        if rc != 0:
            raise RuntimeError(
                f"fqp_solve_batch failed ({self.lib.fqp_error_string(rc).decode()}):"
                f" {self.lib.fqp_last_error(self.h).decode()}")
        self._last_shape = (m, n, P.k)
        self._last_keep = (P, out)        # buffers the adjoint reads
        # the handle keeps the state of its last solve only: a backward
        # through an earlier solve must notice that it was replaced
        self.generation = getattr(self, "generation", 0) + 1
        return out

    def adjoint(self, dL_dw: torch.Tensor, stream=None, noalloc: bool = False, out=None):
        """dL/dmu [m, n] and dL/dB [n, k] (float64) of a loss with gradient
        dL_dw through the last solve on this handle.  noalloc: the entry
        point that allocates no device memory (its scratch is a static
        device array); out = (dmu, dB) reuses the caller's output tensors."""
        if not hasattr(self, "_last_shape"):
            raise RuntimeError("adjoint() needs a preceding solve()")
        m, n, k = self._last_shape
        dev = dL_dw.device
        g = dL_dw.detach().to(torch.float64).contiguous()
        if out is None:
            dmu = torch.empty((m, n), dtype=torch.float64, device=dev)
            dB = torch.empty((n, k), dtype=torch.float64, device=dev)
        else:
            dmu, dB = out
            if dmu.shape != (m, n) or dB.shape != (n, k) or dmu.dtype != torch.float64 \
                    or dB.dtype != torch.float64 or not (dmu.is_contiguous() and dB.is_contiguous()):
                raise ValueError("out must be contiguous float64 tensors of shapes [m, n], [n, k]")
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        fn = self.lib.fqp_adjoint_batch_noalloc if noalloc else self.lib.fqp_adjoint_batch
        rc = fn(self.h, _ptr(g), _ptr(dmu), _ptr(dB), ctypes.c_void_p(stream.cuda_stream))
        if rc != 0:
            name = "fqp_adjoint_batch_noalloc" if noalloc else "fqp_adjoint_batch"
            raise RuntimeError(f"{name} failed ({rc}): "
                               f"{self.lib.fqp_last_error(self.h).decode()}")
        return dmu, dB

    def stats(self) -> dict:
        st = _lib.Stats()
        self.lib.fqp_get_stats(self.h, ctypes.byref(st))
        out = {name: getattr(st, name) for name, _ in _lib.Stats._fields_}
        out["phase_ms"] = [float(x) for x in st.phase_ms]
        return out

    def pass_times(self) -> list:
        """[(ADMM iterations before the pass, ms from the call's start to the
        end of the pass)] for the certification passes of the last solve."""
        count = ctypes.c_int32(0)
        self.lib.fqp_get_pass_times(self.h, None, None, 0, ctypes.byref(count))
        n = count.value
        it = (ctypes.c_int32 * max(n, 1))()
        ms = (ctypes.c_double * max(n, 1))()
        self.lib.fqp_get_pass_times(self.h, it, ms, n, ctypes.byref(count))
        return [(int(it[p]), float(ms[p])) for p in range(n)]


def solve_batch(P: DeviceProblem, solver: Optional[Solver] = None, **settings):
    """One-shot convenience wrapper: returns (outputs, stats)."""
    s = solver or Solver(P.mu.device.index or 0)
    out = s.solve(P, **settings)
    return out, s.stats()


class FqpFunction(torch.autograd.Function):
    """w = argmin of the build's Eq. 1 instance for every account, as a
    differentiable function of the returns mu [m, n] and the factor loadings
    B [n, k]; backward runs the KKT adjoint kernels (dL/dmu, dL/dB)."""

    @staticmethod
    def forward(ctx, mu, B, problem, solver, settings):
        from dataclasses import replace
        P = replace(problem, mu=mu.detach().to(torch.float32).contiguous(),
                    B=B.detach().to(torch.float32).contiguous())
        out = solver.solve(P, **settings)
        ctx.solver = solver
        ctx.generation = solver.generation
        ctx.keep = (P, out)
        ctx.dtypes = (mu.dtype, B.dtype)
        return out["w"].clone()

    @staticmethod
    def backward(ctx, grad_w):
        if ctx.solver.generation != ctx.generation:
            raise RuntimeError(
                "FqpFunction.backward: the Solver has solved another book since this "
                "forward (the adjoint differentiates the handle's last solve only); use "
                "one Solver per differentiable call, or run backward before the next solve")
        dmu, dB = ctx.solver.adjoint(grad_w)
        return dmu.to(ctx.dtypes[0]), dB.to(ctx.dtypes[1]), None, None, None


def solve_differentiable(mu, B, problem: DeviceProblem, solver: Solver,
                         **settings):
    """Autograd entry: weights of every account as a function of (mu, B)."""
    return FqpFunction.apply(mu, B, problem, solver, settings)
