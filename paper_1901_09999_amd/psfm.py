"""Python binding of the HIP library ``libpsfm.so`` (C interface in
``include/psfm.h``).

This module only marshals arguments: torch tensors supply device memory and
the current HIP stream; every step of the computation runs in the library's
kernels.  Importing it on a machine without the built library raises.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpsfm.so")

MAX_GAUSS = 8
STAMP_INVALID, STAMP_REJECTED, STAMP_NONFINITE, STAMP_EXCLUDED, STAMP_PRIOR = 1, 2, 4, 8, 16
MASK_BAD, MASK_CONV_BAD, MASK_CONV_POOR = 1, 2, 4
PREC_FP32, PREC_BF16, PREC_FP16 = 0, 1, 2
WEIGHT_V2, WEIGHT_V1V2 = 0, 1     # fit weights 1 / V2 or 1 / (V1 + V2)
SYNC = 1                          # config flag: solves wait and return the device status


class PsfmError(RuntimeError):
    pass


class CConfig(C.Structure):
    _fields_ = [
        ("n_gauss", C.c_int),
        ("sigma", C.c_double * MAX_GAUSS),
        ("degree", C.c_int * MAX_GAUSS),
        ("half_width", C.c_int),
        ("spatial_order", C.c_int),
        ("stamp_half", C.c_int),
        ("patch", C.c_int),
        ("clip_sigma", C.c_double),
        ("max_iter", C.c_int),
        ("min_stamps", C.c_int),
        ("bad_frac", C.c_double),
        ("precision", C.c_int),
        ("refine", C.c_int),
        ("weight_mode", C.c_int),
        ("ortho_basis", C.c_int),
        ("flags", C.c_int),
        ("fit_band_rows", C.c_int),
    ]


class CStats(C.Structure):
    _fields_ = [
        ("chi2", C.c_double),
        ("dof", C.c_double),
        ("chi2_dof", C.c_double),
        ("kernel_sum_centre", C.c_double),
        ("cov_discarded_frac", C.c_double),
        ("n_used", C.c_int),
        ("n_rejected", C.c_int),
        ("n_iter", C.c_int),
        ("info", C.c_int),
        ("chi2_dof_prior", C.c_double),
        ("n_prior", C.c_int),
        ("n_restored", C.c_int),
        ("n_trusted", C.c_int),
        ("prior_fallback", C.c_int),
        ("n_replaced", C.c_int),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


STATS_BYTES = C.sizeof(CStats)

STAMP_RESERVE = 32
CUT_FEW_STAMPS, CUT_MEAN_DEV, CUT_RMS_DEV, CUT_MOMENT1, CUT_MOMENT2, CUT_DECONV = 1, 2, 4, 8, 16, 32


class CQuality(C.Structure):
    _fields_ = [
        ("dev_mean", C.c_double),
        ("dev_rms", C.c_double),
        ("kernel_sum", C.c_double),
        ("mom_x", C.c_double),
        ("mom_y", C.c_double),
        ("mom_xx", C.c_double),
        ("mom_yy", C.c_double),
        ("deconv_max", C.c_double),
        ("n_used", C.c_int),
        ("cut_flags", C.c_int),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


QUALITY_BYTES = C.sizeof(CQuality)


class CPair(C.Structure):
    _fields_ = [
        ("I1", C.c_void_p), ("V1", C.c_void_p), ("M1", C.c_void_p),
        ("I2", C.c_void_p), ("V2", C.c_void_p), ("M2", C.c_void_p),
        ("width", C.c_int), ("height", C.c_int), ("pitch", C.c_int64),
        ("stamp_xy", C.c_void_p), ("n_stamps", C.c_int), ("spatial_order", C.c_int),
        ("cov1", C.c_void_p), ("cov1_half", C.c_int),
        ("cov2", C.c_void_p), ("cov2_half", C.c_int),
        ("coeffs", C.c_void_p), ("stats", C.c_void_p),
        ("diff", C.c_void_p), ("diff_var", C.c_void_p), ("diff_mask", C.c_void_p),
        ("cov_conv", C.c_void_p), ("cov_conv_half", C.c_int),
        ("cov_diff", C.c_void_p), ("cov_diff_half", C.c_int),
        ("conv", C.c_void_p), ("conv_var", C.c_void_p), ("conv_mask", C.c_void_p),
        ("stamp_flags", C.c_void_p), ("stamp_chi2", C.c_void_p),
    ]


class CTuning(C.Structure):
    _fields_ = [("apply_grid", C.c_int), ("order", C.c_int)]


_lib = None


def lib():
    """Load ``libpsfm.so``; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise PsfmError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        P, i, i64, sz = C.c_void_p, C.c_int, C.c_int64, C.c_size_t
        cp = C.POINTER(CConfig)
        sig = {
            "psfm_config_default": (None, [cp]),
            "psfm_create": (i, [cp, C.POINTER(P)]),
            "psfm_destroy": (i, [P]),
            "psfm_n_basis": (i, [P]),
            "psfm_n_spatial": (i, [P]),
            "psfm_n_unknowns": (i, [P]),
            "psfm_stamp_dim": (i, [P]),
            "psfm_workspace_bytes": (sz, [P, i, i, i]),
            "psfm_stamp_design_floats": (sz, [P, i]),
            "psfm_fit_stamps": (i, [P, P, P, P, P, P, P, i, i, i64, P, i, P, P, P, P, P, P, P, sz, P]),
            "psfm_solve": (i, [P, i, i, P, i, P, P, P, P, P, P, P, P, P, P, sz, P]),
            "psfm_convolve_image": (i, [P, P, P, P, i, i, i64, P, P, P, sz, P]),
            "psfm_propagate_variance": (i, [P, P, P, P, i, i, i64, P, i, P, P, i, P, P, sz, P]),
            "psfm_convolve_pair": (i, [P, P, P, P, P, i, i, i64, P, i, P, P, P, P, i, P, P, sz, P]),
            "psfm_subtract": (i, [P, P, P, P, P, P, P, P, i, i, i64, P, i, P, i, P, P, P, P, i, P,
                                  sz, P]),
            "psfm_match_pair": (i, [P, P, P, P, P, P, P, P, i, i, i64, P, i, P, i, P, P, P, P, i,
                                    P, P, P, P, i, P, P, sz, P]),
            "psfm_match_pair_static": (i, [P, P, P, P, P, P, P, P, i, i, i64, P, i, P, i, P, P, P,
                                           P, i, P, P, P, P, i, P, P]),
            "psfm_fit_norm": (i, [P, P, P, i, i, i64, P, i, P, P, P]),
            "psfm_solve_norm": (i, [P, i, i, P, i, P, P, P, P, P, P, P, P, P, P, P, sz, P]),
            "psfm_quality_eval": (i, [P, P, P, P, P, i, i, i64, P, i, P, C.c_double, P, P, P]),
            "psfm_bin_image": (i, [P, P, P, i, i, i64, i, P, i, P, P, P, i64, P, i, P, P]),
            "psfm_resample_cov": (i, [P, i, C.c_double, P, i, P]),
            "psfm_add_images": (i, [C.c_double, P, P, P, P, i, C.c_double, P, P, P, P, i, i, i, i64, P,
                                    P, P, P, i, P, sz, P]),
            "psfm_dual_workspace_bytes": (sz, [P, i, i, i]),
            "psfm_dual_unknowns": (i, [P]),
            "psfm_fit_dual": (i, [P, P, P, P, P, P, P, i, i, i64, P, i, P, P, P, P, P, P, sz, P]),
            "psfm_solve_dual": (i, [P, i, i, P, i, P, P, P, P, P, C.c_double, P, P, P, P, sz, P]),
            "psfm_dual_subtract": (i, [P, P, P, P, P, P, P, P, i, i, i64, P, P, P, P]),
            "psfm_envelope_psf": (i, [P, i, i, P, P, P]),
            "psfm_render_workspace_bytes": (sz, [i, i, i, C.c_double]),
            "psfm_render_target": (i, [P, i, C.c_double, i, i, i64, P, P, sz, P]),
            "psfm_stack_reject": (i, [i, P, P, P, i64, i, i, i64, C.c_double, P, P]),
            "psfm_trace_mask": (i, [P, P, P, i, i, i64, C.c_double, P, P]),
            "psfm_stack_combine": (i, [i, P, P, P, i64, i, i, i64, P, i, P, P, P, P, P, P, sz, P]),
            "psfm_status_string": (C.c_char_p, [i]),
            "psfm_batch_workspace_bytes": (sz, [P, C.POINTER(CPair), i]),
            "psfm_batch_plan": (i, [P, C.POINTER(CPair), i, C.POINTER(CTuning), P, sz, P, P,
                                    C.POINTER(P)]),
            "psfm_batch_run": (i, [P, P]),
            "psfm_batch_run_stage": (i, [P, i, P]),
            "psfm_batch_set_tuning": (i, [P, C.POINTER(CTuning)]),
            "psfm_batch_graph_capture": (i, [P, P]),
            "psfm_batch_graph_launch": (i, [P, P]),
            "psfm_batch_destroy": (i, [P]),
            "psfm_batch_group_capture": (i, [C.POINTER(P), i, P, C.POINTER(P)]),
            "psfm_batch_group_launch": (i, [P, P]),
            "psfm_batch_group_destroy": (i, [P]),
            "psfm_wall_clock_hz": (C.c_double, []),
            "psfm_solve_stamps": (i, [P, i, P, P, P, P, P, P, P]),
            "psfm_cholesky_workspace_bytes": (sz, [i]),
            "psfm_cholesky_solve": (i, [i, P, P, P, P, P, sz, P]),
            "psfm_solve_prior": (i, [P, i, i, P, i, P, P, P, P, P, P, P, P, P, P, P, sz, P]),
            "psfm_cnn_param_count": (sz, []),
            "psfm_cnn_workspace_bytes": (sz, [i]),
            "psfm_cnn_forward": (i, [P, P, i, P, P, sz, P]),
            "psfm_cnn_loss_grad": (i, [P, P, P, P, i, P, P, P, sz, P]),
            "psfm_cnn_loss_weights": (i, [P, P, P, P, i, P, P]),
            "psfm_cnn_adam": (i, [P, P, P, P, P, sz, i, C.c_float, C.c_float, C.c_float, C.c_float,
                                  P]),
            "psfm_cnn_stamp_inputs": (i, [P, P, P, P, i, i, i64, P, i, P, P, P]),
            "psfm_cnn_targets": (i, [P, P, i, P, P]),
            "psfm_cnn_local_coeffs": (i, [P, P, i, P, P]),
            "psfm_cnn_standardize": (i, [P, P, i, i, P, P, P, P, P]),
            "psfm_cnn_fold_output": (i, [P, P, P, P, P]),
            "psfm_cnn_excess": (i, [P, i, P, P, i, P, P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != 0:
        raise PsfmError(f"{what}: {lib().psfm_status_string(rc).decode()} ({rc})")


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise PsfmError("tensor must live on the HIP device")
    if not t.is_contiguous():
        raise PsfmError("tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


@dataclasses.dataclass
class Config:
    sigmas: Tuple[float, ...] = (0.7, 1.5, 3.0)
    degrees: Tuple[int, ...] = (6, 4, 2)
    h: int = 10
    S: int = 0
    r: int = 20
    P: int = 64
    clip_sigma: float = 3.0
    max_iter: int = 3
    min_stamps: int = 3
    bad_frac: float = 0.2
    precision: int = PREC_FP32
    refine: int = 1
    weight_mode: int = 0          # WEIGHT_V2 or WEIGHT_V1V2
    ortho_basis: int = 0
    flags: int = 0                # SYNC or 0
    fit_band_rows: int = 0        # 0 (from r), 7, 9 or 11

    @classmethod
    def from_workload(cls, wl, **kw):
        base = dict(sigmas=tuple(wl.sigmas), degrees=tuple(wl.degrees), h=wl.kernel_half,
                    S=wl.spatial_order, r=wl.stamp_half, P=wl.patch)
        base.update(kw)
        return cls(**base)

    def c(self) -> CConfig:
        c = CConfig()
        c.n_gauss = len(self.sigmas)
        for j, (s, d) in enumerate(zip(self.sigmas, self.degrees)):
            c.sigma[j] = s
            c.degree[j] = d
        c.half_width, c.spatial_order, c.stamp_half, c.patch = self.h, self.S, self.r, self.P
        c.clip_sigma, c.max_iter, c.min_stamps = self.clip_sigma, self.max_iter, self.min_stamps
        c.bad_frac, c.precision, c.refine = self.bad_frac, self.precision, self.refine
        c.weight_mode, c.ortho_basis = self.weight_mode, self.ortho_basis
        c.flags, c.fit_band_rows = self.flags, self.fit_band_rows
        return c


class Context:
    """A library context (basis tables on the current device) plus cached
    workspace.  All image arguments are CUDA/HIP torch tensors."""

    def __init__(self, cfg: Config, device: Optional[torch.device] = None):
        self.cfg = cfg
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else device
        self._h = C.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().psfm_create(C.byref(cfg.c()), C.byref(self._h)), "psfm_create")
        self.nb = lib().psfm_n_basis(self._h)
        self.ns = lib().psfm_n_spatial(self._h)
        self.N = lib().psfm_n_unknowns(self._h)
        self.L = lib().psfm_stamp_dim(self._h)
        self._ws: Optional[torch.Tensor] = None

    def close(self):
        if self._h:
            lib().psfm_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def workspace(self, W: int, H: int, n_stamps: int) -> torch.Tensor:
        need = lib().psfm_workspace_bytes(self._h, W, H, n_stamps)
        if need == 0:
            raise PsfmError("invalid workspace request")
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        return self._ws

    # ------------------------------------------------------------------ calls
    def fit_stamps(self, I1, M1, I2, V2, M2, stamps, out=None, V1=None):
        """psfm_fit_stamps (V1 is read with weight_mode WEIGHT_V1V2 only)."""
        H, W = I1.shape
        n = stamps.shape[0]
        L = self.L
        dev = self.device
        if out is None:
            out = dict(M=torch.empty((n, L, L), dtype=torch.float64, device=dev),
                       b=torch.empty((n, L), dtype=torch.float64, device=dev),
                       e=torch.empty(n, dtype=torch.float64, device=dev),
                       npix=torch.empty(n, dtype=torch.int32, device=dev),
                       flags=torch.empty(n, dtype=torch.int32, device=dev),
                       design=self.design_buffer(n))
        ws = self.workspace(W, H, n)
        _check(lib().psfm_fit_stamps(self._h, _ptr(I1), _ptr(V1), _ptr(M1), _ptr(I2), _ptr(V2),
                                     _ptr(M2), W, H, W, _ptr(stamps), n, _ptr(out["M"]), _ptr(out["b"]),
                                     _ptr(out["e"]), _ptr(out["npix"]), _ptr(out["flags"]),
                                     _ptr(out.get("design")), _ptr(ws), ws.numel(), _stream()),
               "psfm_fit_stamps")
        return out

    def design_buffer(self, n):
        """FP32 stamp design of the 16-bit modes (None in FP32)."""
        k = lib().psfm_stamp_design_floats(self._h, n)
        return torch.empty(k, dtype=torch.float32, device=self.device) if k else None

    def solve_stamps(self, fit):
        """Each stamp's own least-squares kernel: (local [n, L], chi2 [n])."""
        n = fit["M"].shape[0]
        local = torch.empty((n, self.L), dtype=torch.float64, device=self.device)
        chi2 = torch.empty(max(n, 1), dtype=torch.float64, device=self.device)
        _check(lib().psfm_solve_stamps(self._h, n, _ptr(fit["M"]), _ptr(fit["b"]), _ptr(fit["e"]),
                                       _ptr(fit["flags"]), _ptr(local), _ptr(chi2), _stream()),
               "psfm_solve_stamps")
        return local, chi2[:n]

    def solve(self, W, H, stamps, fit, flags=None, out=None, prior=None, flags_inplace=False):
        """psfm_solve, or psfm_solve_prior when ``prior`` (n x L float64
        predicted local coefficients) is given.  The stamp flags are updated
        in a copy, or in ``flags`` itself with ``flags_inplace``."""
        n = stamps.shape[0]
        dev = self.device
        if flags_inplace and flags is not None:
            fl = flags
        else:
            fl = (fit["flags"] if flags is None else flags).clone()
        if out is None:
            out = dict(coeffs=torch.empty(self.N, dtype=torch.float64, device=dev),
                       chi2=torch.empty(max(n, 1), dtype=torch.float64, device=dev),
                       stats=torch.zeros(STATS_BYTES, dtype=torch.uint8, device=dev))
        out["flags"] = fl
        ws = self.workspace(W, H, n)
        if prior is not None:
            _check(lib().psfm_solve_prior(self._h, W, H, _ptr(stamps), n, _ptr(fit["M"]), _ptr(fit["b"]),
                                          _ptr(fit["e"]), _ptr(fit["npix"]), _ptr(fl),
                                          _ptr(fit.get("design")), _ptr(prior), _ptr(out["coeffs"]),
                                          _ptr(out["chi2"]), _ptr(out["stats"]), _ptr(ws), ws.numel(),
                                          _stream()), "psfm_solve_prior")
            return out
        _check(lib().psfm_solve(self._h, W, H, _ptr(stamps), n, _ptr(fit["M"]), _ptr(fit["b"]),
                                _ptr(fit["e"]), _ptr(fit["npix"]), _ptr(fl), _ptr(fit.get("design")),
                                _ptr(out["coeffs"]),
                                _ptr(out["chi2"]), _ptr(out["stats"]), _ptr(ws), ws.numel(),
                                _stream()), "psfm_solve")
        return out

    # ------------------------------------------- the paper's normalisation mode
    def fit_norm(self, I1, I2, stamps, flags, out=None):
        """psfm_fit_norm: per-stamp unweighted sums [n, 5] (npix, sum A0,
        sum I2, sum A0^2, sum A0 I2)."""
        H, W = I1.shape
        n = stamps.shape[0]
        out = torch.empty((max(n, 1), 5), dtype=torch.float64, device=self.device) if out is None else out
        _check(lib().psfm_fit_norm(self._h, _ptr(I1), _ptr(I2), W, H, W, _ptr(stamps), n, _ptr(flags),
                                   _ptr(out), _stream()), "psfm_fit_norm")
        return out[:n]

    def solve_norm(self, W, H, stamps, fit, norm, flags=None, group=None, out=None):
        """psfm_solve_norm (b0, d0 from stamp totals, held; replacement from
        ``group`` reserves).  Stamp flags are updated in a copy."""
        n = stamps.shape[0]
        dev = self.device
        fl = (fit["flags"] if flags is None else flags).clone()
        if out is None:
            out = dict(coeffs=torch.empty(self.N, dtype=torch.float64, device=dev),
                       chi2=torch.empty(max(n, 1), dtype=torch.float64, device=dev),
                       stats=torch.zeros(STATS_BYTES, dtype=torch.uint8, device=dev))
        out["flags"] = fl
        ws = self.workspace(W, H, n)
        _check(lib().psfm_solve_norm(self._h, W, H, _ptr(stamps), n, _ptr(fit["M"]), _ptr(fit["b"]),
                                     _ptr(fit["e"]), _ptr(fit["npix"]), _ptr(norm), _ptr(group), _ptr(fl),
                                     _ptr(out["coeffs"]), _ptr(out["chi2"]), _ptr(out["stats"]), _ptr(ws),
                                     ws.numel(), _stream()), "psfm_solve_norm")
        return out

    def quality(self, coeffs, I1, I2, V2, stamps, flags, soft=0.0):
        """psfm_quality_eval: (quality tensor, per-stamp deviations)."""
        H, W = I1.shape
        n = stamps.shape[0]
        dev = torch.empty(max(n, 1), dtype=torch.float64, device=self.device)
        q = torch.zeros(QUALITY_BYTES, dtype=torch.uint8, device=self.device)
        _check(lib().psfm_quality_eval(self._h, _ptr(coeffs), _ptr(I1), _ptr(I2), _ptr(V2), W, H, W,
                                       _ptr(stamps), n, _ptr(flags), float(soft), _ptr(dev), _ptr(q),
                                       _stream()), "psfm_quality_eval")
        return q, dev[:n]

    # ------------------------------------------------- both images to a common PSF
    @property
    def N2(self) -> int:
        return lib().psfm_dual_unknowns(self._h)

    def dual_workspace(self, W: int, H: int, n_stamps: int) -> torch.Tensor:
        need = lib().psfm_dual_workspace_bytes(self._h, W, H, n_stamps)
        if need == 0:
            raise PsfmError("invalid workspace request")
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        return self._ws

    def fit_dual(self, I1, M1, I2, V2, M2, stamps, V1=None):
        """psfm_fit_dual: dict(M [n, 2nb, 2nb], b, e, npix, flags)."""
        H, W = I1.shape
        n = stamps.shape[0]
        L = 2 * self.nb
        dev = self.device
        out = dict(M=torch.empty((n, L, L), dtype=torch.float64, device=dev),
                   b=torch.empty((n, L), dtype=torch.float64, device=dev),
                   e=torch.empty(n, dtype=torch.float64, device=dev),
                   npix=torch.empty(n, dtype=torch.int32, device=dev),
                   flags=torch.empty(n, dtype=torch.int32, device=dev))
        ws = self.dual_workspace(W, H, n)
        _check(lib().psfm_fit_dual(self._h, _ptr(I1), _ptr(V1), _ptr(M1), _ptr(I2), _ptr(V2), _ptr(M2),
                                   W, H, W,
                                   _ptr(stamps), n, _ptr(out["M"]), _ptr(out["b"]), _ptr(out["e"]),
                                   _ptr(out["npix"]), _ptr(out["flags"]), _ptr(ws), ws.numel(),
                                   _stream()), "psfm_fit_dual")
        return out

    def solve_dual(self, W, H, stamps, fit, phi, flags=None):
        """psfm_solve_dual: dict(coeffs [N2], chi2, stats, flags)."""
        n = stamps.shape[0]
        dev = self.device
        fl = (fit["flags"] if flags is None else flags).clone()
        out = dict(coeffs=torch.empty(self.N2, dtype=torch.float64, device=dev),
                   chi2=torch.empty(max(n, 1), dtype=torch.float64, device=dev),
                   stats=torch.zeros(STATS_BYTES, dtype=torch.uint8, device=dev), flags=fl)
        ws = self.dual_workspace(W, H, n)
        _check(lib().psfm_solve_dual(self._h, W, H, _ptr(stamps), n, _ptr(fit["M"]), _ptr(fit["b"]),
                                     _ptr(fit["e"]), _ptr(fit["npix"]), _ptr(fl), float(phi),
                                     _ptr(out["coeffs"]), _ptr(out["chi2"]), _ptr(out["stats"]), _ptr(ws),
                                     ws.numel(), _stream()), "psfm_solve_dual")
        return out

    def dual_subtract(self, coeffs, I1, V1, M1, I2, V2, M2):
        """psfm_dual_subtract: (D, V_D, mask_D)."""
        H, W = I1.shape
        D = torch.empty_like(I1)
        VD = torch.empty_like(V1)
        MD = torch.empty_like(M1)
        _check(lib().psfm_dual_subtract(self._h, _ptr(coeffs), _ptr(I1), _ptr(V1), _ptr(M1), _ptr(I2),
                                        _ptr(V2), _ptr(M2), W, H, W, _ptr(D), _ptr(VD), _ptr(MD),
                                        _stream()), "psfm_dual_subtract")
        return D, VD, MD

    def convolve_image(self, coeffs, I, M, out=None, out_mask=None):
        H, W = I.shape
        out = torch.empty_like(I) if out is None else out
        out_mask = torch.empty_like(M) if out_mask is None else out_mask
        ws = self.workspace(W, H, 0)
        _check(lib().psfm_convolve_image(self._h, _ptr(coeffs), _ptr(I), _ptr(M), W, H, W,
                                         _ptr(out), _ptr(out_mask), _ptr(ws), ws.numel(),
                                         _stream()), "psfm_convolve_image")
        return out, out_mask

    def propagate_variance(self, coeffs, V, M, cov_in=None, c_out=10, stats=None, out=None,
                           cov_out=None):
        H, W = V.shape
        out = torch.empty_like(V) if out is None else out
        if cov_out is None:
            cov_out = torch.empty((2 * c_out + 1, 2 * c_out + 1), dtype=torch.float64,
                                  device=self.device)
        c_in = 0 if cov_in is None else (cov_in.shape[0] - 1) // 2
        ws = self.workspace(W, H, 0)
        _check(lib().psfm_propagate_variance(self._h, _ptr(coeffs), _ptr(V), _ptr(M), W, H, W,
                                             _ptr(cov_in), c_in, _ptr(out), _ptr(cov_out), c_out,
                                             _ptr(stats), _ptr(ws), ws.numel(), _stream()),
               "psfm_propagate_variance")
        return out, cov_out

    def convolve_pair(self, coeffs, I, V, M, cov_in=None, c_out=10, stats=None, out=None,
                      out_mask=None, var_out=None, cov_out=None):
        """psfm_convolve_pair: convolve_image and propagate_variance in one call
        (one patch-kernel realisation per tile); returns (conv, conv_mask, var, cov)."""
        H, W = I.shape
        out = torch.empty_like(I) if out is None else out
        out_mask = torch.empty_like(M) if out_mask is None else out_mask
        var_out = torch.empty_like(V) if var_out is None else var_out
        if cov_out is None:
            cov_out = torch.empty((2 * c_out + 1, 2 * c_out + 1), dtype=torch.float64,
                                  device=self.device)
        c_in = 0 if cov_in is None else (cov_in.shape[0] - 1) // 2
        ws = self.workspace(W, H, 0)
        _check(lib().psfm_convolve_pair(self._h, _ptr(coeffs), _ptr(I), _ptr(V), _ptr(M), W, H, W,
                                        _ptr(cov_in), c_in, _ptr(out), _ptr(out_mask), _ptr(var_out),
                                        _ptr(cov_out), c_out, _ptr(stats), _ptr(ws), ws.numel(),
                                        _stream()), "psfm_convolve_pair")
        return out, out_mask, var_out, cov_out

    def subtract(self, coeffs, I2, V2, M2, conv, conv_var, conv_mask, cov_conv, cov2=None,
                 c_d=None, out=None):
        H, W = I2.shape
        cc = (cov_conv.shape[0] - 1) // 2
        c2 = 0 if cov2 is None else (cov2.shape[0] - 1) // 2
        cd = max(cc, c2) if c_d is None else c_d
        if out is None:
            out = dict(diff=torch.empty_like(I2), diff_var=torch.empty_like(V2),
                       diff_mask=torch.empty_like(M2),
                       cov_diff=torch.empty((2 * cd + 1, 2 * cd + 1), dtype=torch.float64,
                                            device=self.device))
        ws = self.workspace(W, H, 0)
        _check(lib().psfm_subtract(self._h, _ptr(coeffs), _ptr(I2), _ptr(V2), _ptr(M2), _ptr(conv),
                                   _ptr(conv_var), _ptr(conv_mask), W, H, W, _ptr(cov2), c2,
                                   _ptr(cov_conv), cc, _ptr(out["diff"]), _ptr(out["diff_var"]),
                                   _ptr(out["diff_mask"]), _ptr(out["cov_diff"]), cd, _ptr(ws),
                                   ws.numel(), _stream()), "psfm_subtract")
        return out

    def match(self, coeffs, I1, V1, M1, I2, V2, M2, cov1=None, cov2=None, c_out=10, c_d=None,
              stats=None, out=None, cov_conv=None, conv=None, conv_mask=None, conv_var=None):
        """psfm_match_pair: convolve_pair and subtract in one pass over the
        tiles.  The convolved planes are written only into the given
        ``conv``/``conv_mask`` (both or neither) and ``conv_var``; returns the
        subtract dict plus ``cov`` (the convolved image's pseudo-matrix)."""
        H, W = I1.shape
        c1 = 0 if cov1 is None else (cov1.shape[0] - 1) // 2
        c2 = 0 if cov2 is None else (cov2.shape[0] - 1) // 2
        cd = max(c_out, c2) if c_d is None else c_d
        if cov_conv is None:
            cov_conv = torch.empty((2 * c_out + 1, 2 * c_out + 1), dtype=torch.float64,
                                   device=self.device)
        if out is None:
            out = dict(diff=torch.empty_like(I2), diff_var=torch.empty_like(V2),
                       diff_mask=torch.empty_like(M2),
                       cov_diff=torch.empty((2 * cd + 1, 2 * cd + 1), dtype=torch.float64,
                                            device=self.device))
        ws = self.workspace(W, H, 0)
        _check(lib().psfm_match_pair(self._h, _ptr(coeffs), _ptr(I1), _ptr(V1), _ptr(M1), _ptr(I2),
                                     _ptr(V2), _ptr(M2), W, H, W, _ptr(cov1), c1, _ptr(cov2), c2,
                                     _ptr(conv), _ptr(conv_mask), _ptr(conv_var), _ptr(cov_conv),
                                     c_out, _ptr(out["diff"]), _ptr(out["diff_var"]),
                                     _ptr(out["diff_mask"]), _ptr(out["cov_diff"]), cd, _ptr(stats),
                                     _ptr(ws), ws.numel(), _stream()), "psfm_match_pair")
        return dict(out, cov=cov_conv)

    def match_static(self, coeffs, I1, V1, M1, I2, V2, M2, cov1=None, cov2=None, c_out=10,
                     c_d=None, stats=None, out=None, cov_conv=None, conv=None, conv_mask=None,
                     conv_var=None):
        """psfm_match_pair_static: :meth:`match` with the library's static
        device scratch instead of a workspace (the call allocates nothing when
        every output is given)."""
        H, W = I1.shape
        c1 = 0 if cov1 is None else (cov1.shape[0] - 1) // 2
        c2 = 0 if cov2 is None else (cov2.shape[0] - 1) // 2
        cd = max(c_out, c2) if c_d is None else c_d
        if cov_conv is None:
            cov_conv = torch.empty((2 * c_out + 1, 2 * c_out + 1), dtype=torch.float64,
                                   device=self.device)
        if out is None:
            out = dict(diff=torch.empty_like(I2), diff_var=torch.empty_like(V2),
                       diff_mask=torch.empty_like(M2),
                       cov_diff=torch.empty((2 * cd + 1, 2 * cd + 1), dtype=torch.float64,
                                            device=self.device))
        _check(lib().psfm_match_pair_static(
            self._h, _ptr(coeffs), _ptr(I1), _ptr(V1), _ptr(M1), _ptr(I2), _ptr(V2), _ptr(M2), W,
            H, W, _ptr(cov1), c1, _ptr(cov2), c2, _ptr(conv), _ptr(conv_mask), _ptr(conv_var),
            _ptr(cov_conv), c_out, _ptr(out["diff"]), _ptr(out["diff_var"]),
            _ptr(out["diff_mask"]), _ptr(out["cov_diff"]), cd, _ptr(stats), _stream()),
            "psfm_match_pair_static")
        return dict(out, cov=cov_conv)

    def match_pair(self, I1, V1, M1, I2, V2, M2, stamps, c_out=10, bufs=None):
        """The whole hot path: fit -> solve -> convolve -> variance -> subtract.
        ``bufs`` (from :meth:`alloc_pair`) avoids allocations in a timed loop."""
        H, W = I1.shape
        b = self.alloc_pair(W, H, stamps.shape[0], c_out) if bufs is None else bufs
        fit = self.fit_stamps(I1, M1, I2, V2, M2, stamps, out=b["fit"], V1=V1)
        b["flags_in"].copy_(fit["flags"])
        sol = self.solve(W, H, stamps, fit, flags=b["flags_in"], out=b["sol"], flags_inplace=True)
        sub = self.match(sol["coeffs"], I1, V1, M1, I2, V2, M2, c_out=c_out, stats=sol["stats"],
                         out=b["sub"], cov_conv=b["cov"], conv=b["conv"], conv_mask=b["conv_mask"],
                         conv_var=b["var"])
        return dict(fit=fit, sol=sol, conv=b["conv"], conv_mask=b["conv_mask"], var=b["var"], **sub)

    def alloc_pair(self, W, H, n, c_out=10):
        dev, L = self.device, self.L
        f32 = dict(dtype=torch.float32, device=dev)
        return dict(
            fit=dict(M=torch.empty((n, L, L), dtype=torch.float64, device=dev),
                     b=torch.empty((n, L), dtype=torch.float64, device=dev),
                     e=torch.empty(n, dtype=torch.float64, device=dev),
                     npix=torch.empty(n, dtype=torch.int32, device=dev),
                     flags=torch.empty(n, dtype=torch.int32, device=dev),
                     design=self.design_buffer(n)),
            flags_in=torch.empty(n, dtype=torch.int32, device=dev),
            sol=dict(coeffs=torch.empty(self.N, dtype=torch.float64, device=dev),
                     chi2=torch.empty(max(n, 1), dtype=torch.float64, device=dev),
                     stats=torch.zeros(STATS_BYTES, dtype=torch.uint8, device=dev)),
            conv=torch.empty((H, W), **f32), conv_mask=torch.empty((H, W), dtype=torch.uint8, device=dev),
            var=torch.empty((H, W), **f32),
            cov=torch.empty((2 * c_out + 1, 2 * c_out + 1), dtype=torch.float64, device=dev),
            sub=dict(diff=torch.empty((H, W), **f32), diff_var=torch.empty((H, W), **f32),
                     diff_mask=torch.empty((H, W), dtype=torch.uint8, device=dev),
                     cov_diff=torch.empty((2 * c_out + 1, 2 * c_out + 1), dtype=torch.float64,
                                          device=dev)),
        )


class Batch:
    """A planned batch of independent pairs (``psfm_batch_*``).

    ``pairs`` is a sequence of dicts with device tensors I1, V1, M1, I2, V2,
    M2, stamps and an int ``S`` (spatial order), optionally ``cov1`` /
    ``cov2``.  Outputs are allocated here, once; :meth:`run` launches the
    whole batch, :meth:`capture` / :meth:`launch` go through one HIP graph.
    ``keep_conv`` also writes I', V' and their mask per pair.
    """

    def __init__(self, ctx: Context, pairs, c_out: int = 10, keep_conv: bool = False,
                 apply_grid: int = 0, order: int = 0, stream: Optional[torch.cuda.Stream] = None):
        self.ctx = ctx
        dev = ctx.device
        self.stream = torch.cuda.Stream(device=dev) if stream is None else stream
        self.n = len(pairs)
        self.inputs = list(pairs)
        self.out = []
        cp = (CPair * self.n)()
        f32 = dict(dtype=torch.float32, device=dev)
        for k, q in enumerate(pairs):
            H, W = q["I1"].shape
            S = int(q["S"])
            ns = (S + 1) * (S + 2) // 2
            N = ctx.nb * ns + 1
            n = q["stamps"].shape[0]
            cov1, cov2 = q.get("cov1"), q.get("cov2")
            c2 = 0 if cov2 is None else (cov2.shape[0] - 1) // 2
            cd = max(c_out, c2)
            o = dict(coeffs=torch.zeros(N, dtype=torch.float64, device=dev),
                     stats=torch.zeros(STATS_BYTES, dtype=torch.uint8, device=dev),
                     diff=torch.empty((H, W), **f32), diff_var=torch.empty((H, W), **f32),
                     diff_mask=torch.empty((H, W), dtype=torch.uint8, device=dev),
                     cov=torch.empty((2 * c_out + 1,) * 2, dtype=torch.float64, device=dev),
                     cov_diff=torch.empty((2 * cd + 1,) * 2, dtype=torch.float64, device=dev),
                     flags=torch.empty(max(n, 1), dtype=torch.int32, device=dev),
                     chi2=torch.empty(max(n, 1), dtype=torch.float64, device=dev))
            if keep_conv:
                o.update(conv=torch.empty((H, W), **f32), var=torch.empty((H, W), **f32),
                         conv_mask=torch.empty((H, W), dtype=torch.uint8, device=dev))
            self.out.append(o)
            c = cp[k]
            c.I1, c.V1, c.M1 = _ptr(q["I1"]), _ptr(q["V1"]), _ptr(q["M1"])
            c.I2, c.V2, c.M2 = _ptr(q["I2"]), _ptr(q["V2"]), _ptr(q["M2"])
            c.width, c.height, c.pitch = W, H, W
            c.stamp_xy, c.n_stamps, c.spatial_order = _ptr(q["stamps"]), n, S
            c.cov1, c.cov1_half = _ptr(cov1), 0 if cov1 is None else (cov1.shape[0] - 1) // 2
            c.cov2, c.cov2_half = _ptr(cov2), c2
            c.coeffs, c.stats = _ptr(o["coeffs"]), _ptr(o["stats"])
            c.diff, c.diff_var, c.diff_mask = _ptr(o["diff"]), _ptr(o["diff_var"]), _ptr(o["diff_mask"])
            c.cov_conv, c.cov_conv_half = _ptr(o["cov"]), c_out
            c.cov_diff, c.cov_diff_half = _ptr(o["cov_diff"]), cd
            if keep_conv:
                c.conv, c.conv_var, c.conv_mask = _ptr(o["conv"]), _ptr(o["var"]), _ptr(o["conv_mask"])
            c.stamp_flags, c.stamp_chi2 = _ptr(o["flags"]), _ptr(o["chi2"])
        self._cpairs = cp
        need = lib().psfm_batch_workspace_bytes(ctx.handle, cp, self.n)
        if need == 0:
            raise PsfmError("invalid batch")
        self.ws = torch.empty(need, dtype=torch.uint8, device=dev)
        self.times = torch.zeros(self.n + 1, dtype=torch.int64, device=dev)
        self._h = C.c_void_p()
        tu = CTuning(apply_grid, order)
        with torch.cuda.stream(self.stream):
            _check(lib().psfm_batch_plan(ctx.handle, cp, self.n, C.byref(tu), _ptr(self.ws),
                                         self.ws.numel(), _ptr(self.times), _stream(),
                                         C.byref(self._h)), "psfm_batch_plan")
        self.tick_hz = lib().psfm_wall_clock_hz()

    def close(self):
        if self._h:
            lib().psfm_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_apply_grid(self, grid: int):
        _check(lib().psfm_batch_set_tuning(self._h, C.byref(CTuning(grid, 0))), "psfm_batch_set_tuning")

    def run(self):
        """Launch the batch on the batch stream (ordered after the current stream)."""
        self.stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(self.stream):
            _check(lib().psfm_batch_run(self._h, _stream()), "psfm_batch_run")
        torch.cuda.current_stream().wait_stream(self.stream)

    def run_stage(self, stage: int):
        """One stage (0 fit, 1 solve, 2 patch kernels and pseudo-matrices,
        3 fused convolution / difference pass) on the current stream."""
        _check(lib().psfm_batch_run_stage(self._h, stage, _stream()), "psfm_batch_run_stage")

    def capture(self):
        torch.cuda.synchronize()
        with torch.cuda.stream(self.stream):
            _check(lib().psfm_batch_graph_capture(self._h, _stream()), "psfm_batch_graph_capture")

    def launch(self):
        self.stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(self.stream):
            _check(lib().psfm_batch_graph_launch(self._h, _stream()), "psfm_batch_graph_launch")
        torch.cuda.current_stream().wait_stream(self.stream)

    def latencies_s(self) -> np.ndarray:
        """Completion time of each pair after the start of the last run (s)."""
        t = self.times.cpu().numpy().astype(np.uint64)
        return (t[1:] - t[0]).astype(np.float64) / self.tick_hz

    def stats(self, k: int) -> dict:
        return read_stats(self.out[k]["stats"])


def split_by_order(pairs, groups) -> List[List[int]]:
    """Indices of the pairs whose spatial order ``S`` lies in each group of
    orders (a sequence of sequences); pairs of no listed order form a last
    group.  Empty groups are dropped."""
    listed = {int(s) for g in groups for s in g}
    out = [[k for k, q in enumerate(pairs) if int(q["S"]) in set(int(s) for s in g)] for g in groups]
    out.append([k for k, q in enumerate(pairs) if int(q["S"]) not in listed])
    return [ix for ix in out if ix]


class BatchGroup:
    """Several :class:`Batch` plans as the branches of one HIP graph
    (``psfm_batch_group_*``): each plan's run is forked from and joined back
    to the group's stream, so that one plan's latency-bound solve overlaps
    another's fits or tile pass.  The group holds the plans (which must not
    run by themselves while it runs)."""

    def __init__(self, batches, stream: Optional[torch.cuda.Stream] = None):
        self.batches = list(batches)
        if not self.batches:
            raise PsfmError("empty batch group")
        dev = self.batches[0].ctx.device
        self.stream = torch.cuda.Stream(device=dev) if stream is None else stream
        self._h = C.c_void_p()
        arr = (C.c_void_p * len(self.batches))(*[b._h.value for b in self.batches])
        torch.cuda.synchronize()
        with torch.cuda.stream(self.stream):
            _check(lib().psfm_batch_group_capture(arr, len(self.batches), _stream(), C.byref(self._h)),
                   "psfm_batch_group_capture")

    def launch(self):
        self.stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(self.stream):
            _check(lib().psfm_batch_group_launch(self._h, _stream()), "psfm_batch_group_launch")
        torch.cuda.current_stream().wait_stream(self.stream)

    def close(self):
        if self._h:
            lib().psfm_batch_group_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cholesky_solve(M: torch.Tensor, b: torch.Tensor, x: Optional[torch.Tensor] = None,
                   info: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None):
    """psfm_cholesky_solve on device tensors (M n x n, b n, float64)."""
    n = b.numel()
    x = torch.empty_like(b) if x is None else x
    info = torch.zeros(1, dtype=torch.int32, device=b.device) if info is None else info
    if ws is None:
        ws = torch.empty(int(lib().psfm_cholesky_workspace_bytes(n)), dtype=torch.uint8, device=b.device)
    _check(lib().psfm_cholesky_solve(n, _ptr(M), _ptr(b), _ptr(x), _ptr(info), _ptr(ws), ws.numel(),
                                     _stream()), "psfm_cholesky_solve")
    return x, info


ADD_WORKSPACE_BYTES = 32768


def bin_image(I, V, M, B, cov_in=None, c_out=4):
    """psfm_bin_image: (Ib, Vb, Mb, cov_b, discarded) on the device."""
    H, W = I.shape
    Wb, Hb = W // B, H // B
    dev = I.device
    Ib = torch.empty((Hb, Wb), dtype=torch.float32, device=dev)
    Vb = torch.empty((Hb, Wb), dtype=torch.float32, device=dev)
    Mb = torch.empty((Hb, Wb), dtype=torch.uint8, device=dev)
    cov = torch.empty((2 * c_out + 1, 2 * c_out + 1), dtype=torch.float64, device=dev)
    disc = torch.zeros(1, dtype=torch.float64, device=dev)
    c_in = 0 if cov_in is None else (cov_in.shape[0] - 1) // 2
    _check(lib().psfm_bin_image(_ptr(I), _ptr(V), _ptr(M), W, H, W, B, _ptr(cov_in), c_in, _ptr(Ib),
                                _ptr(Vb), _ptr(Mb), Wb, _ptr(cov), c_out, _ptr(disc), _stream()),
           "psfm_bin_image")
    return Ib, Vb, Mb, cov, disc


def resample_cov(cov_in, scale, c_out):
    out = torch.empty((2 * c_out + 1, 2 * c_out + 1), dtype=torch.float64, device=cov_in.device)
    _check(lib().psfm_resample_cov(_ptr(cov_in), (cov_in.shape[0] - 1) // 2, float(scale), _ptr(out),
                                   c_out, _stream()), "psfm_resample_cov")
    return out


def add_images(alpha, Ia, Va, Ma, cov_a, beta, Ib, Vb, Mb, cov_b, cs, out=None, ws=None):
    """psfm_add_images: dict(S, VS, MS, cov)."""
    H, W = Ia.shape
    dev = Ia.device
    if out is None:
        out = dict(S=torch.empty_like(Ia), VS=torch.empty_like(Va), MS=torch.empty_like(Ma),
                   cov=torch.empty((2 * cs + 1, 2 * cs + 1), dtype=torch.float64, device=dev))
    ws = torch.empty(ADD_WORKSPACE_BYTES, dtype=torch.uint8, device=dev) if ws is None else ws
    ca = 0 if cov_a is None else (cov_a.shape[0] - 1) // 2
    cb = 0 if cov_b is None else (cov_b.shape[0] - 1) // 2
    _check(lib().psfm_add_images(float(alpha), _ptr(Ia), _ptr(Va), _ptr(Ma), _ptr(cov_a), ca, float(beta),
                                 _ptr(Ib), _ptr(Vb), _ptr(Mb), _ptr(cov_b), cb, W, H, W, _ptr(out["S"]),
                                 _ptr(out["VS"]), _ptr(out["MS"]), _ptr(out["cov"]), cs, _ptr(ws),
                                 ws.numel(), _stream()), "psfm_add_images")
    return out


STACK_WORKSPACE_BYTES = 262656
STACK_MAX_INPUTS = 64


def envelope_psf(params, half):
    """psfm_envelope_psf: params (n, 3) float64 (sigma_major, sigma_minor,
    angle) on the device -> (sigma (1,), env (2 half + 1)^2)."""
    dev = params.device
    env = torch.empty((2 * half + 1, 2 * half + 1), dtype=torch.float64, device=dev)
    sig = torch.empty(1, dtype=torch.float64, device=dev)
    _check(lib().psfm_envelope_psf(_ptr(params), params.shape[0], half, _ptr(env), _ptr(sig), _stream()),
           "psfm_envelope_psf")
    return sig, env


def render_target(src, sigma, W, H, out=None, ws=None):
    """psfm_render_target: src (n, 3) float64 (x, y, flux) on the device."""
    n = src.shape[0]
    dev = src.device
    need = int(lib().psfm_render_workspace_bytes(n, W, H, float(sigma)))
    if need == 0:
        raise PsfmError("psfm_render_workspace_bytes: invalid arguments")
    out = torch.empty((H, W), dtype=torch.float32, device=dev) if out is None else out
    ws = torch.empty(need, dtype=torch.uint8, device=dev) if ws is None else ws
    _check(lib().psfm_render_target(_ptr(src), n, float(sigma), W, H, W, _ptr(out), _ptr(ws), ws.numel(),
                                    _stream()), "psfm_render_target")
    return out


def stack_reject(I, V, M, nsigma, out=None):
    """psfm_stack_reject on (n, H, W) planes."""
    n, H, W = I.shape
    out = torch.empty_like(M) if out is None else out
    _check(lib().psfm_stack_reject(n, _ptr(I), _ptr(V), _ptr(M), H * W, W, H, W, float(nsigma), _ptr(out),
                                   _stream()), "psfm_stack_reject")
    return out


def trace_mask(ctx, coeffs, outliers, frac, out=None):
    """psfm_trace_mask: the input pixels behind the outliers of a convolved image."""
    H, W = outliers.shape
    out = torch.empty_like(outliers) if out is None else out
    _check(lib().psfm_trace_mask(ctx.handle, _ptr(coeffs), _ptr(outliers), W, H, W, float(frac), _ptr(out),
                                 _stream()), "psfm_trace_mask")
    return out


def stack_combine(I, V, M, cov=None, out=None, ws=None):
    """psfm_stack_combine on (n, H, W) planes; cov (n, 2c + 1, 2c + 1) or
    None.  Returns dict(S, VS, MS, cov, weights)."""
    n, H, W = I.shape
    dev = I.device
    ck = 0 if cov is None else (cov.shape[1] - 1) // 2
    if out is None:
        out = dict(S=torch.empty((H, W), dtype=torch.float32, device=dev),
                   VS=torch.empty((H, W), dtype=torch.float32, device=dev),
                   MS=torch.empty((H, W), dtype=torch.uint8, device=dev),
                   cov=None if cov is None else torch.empty((2 * ck + 1,) * 2, dtype=torch.float64,
                                                            device=dev),
                   weights=torch.empty(n, dtype=torch.float64, device=dev))
    ws = torch.empty(STACK_WORKSPACE_BYTES, dtype=torch.uint8, device=dev) if ws is None else ws
    _check(lib().psfm_stack_combine(n, _ptr(I), _ptr(V), _ptr(M), H * W, W, H, W, _ptr(cov), ck,
                                    _ptr(out["S"]), _ptr(out["VS"]), _ptr(out["MS"]), _ptr(out["cov"]),
                                    _ptr(out["weights"]), _ptr(ws), ws.numel(), _stream()),
           "psfm_stack_combine")
    return out


def read_quality(q: torch.Tensor) -> dict:
    raw = bytes(q.cpu().numpy().tobytes())
    return CQuality.from_buffer_copy(raw[:QUALITY_BYTES]).as_dict()


def read_stats(stats: torch.Tensor) -> dict:
    raw = bytes(stats.cpu().numpy().tobytes())
    return CStats.from_buffer_copy(raw[:STATS_BYTES]).as_dict()


def to_device(pair, device="cuda"):
    """Upload a synthetic pair's planes and stamp list."""
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
    return dict(I1=t(pair.I1), V1=t(pair.V1), M1=t(pair.M1), I2=t(pair.I2), V2=t(pair.V2),
                M2=t(pair.M2), stamps=t(pair.stamps.astype(np.int32)))


def exported_symbols() -> Sequence[str]:
    return ["psfm_config_default", "psfm_create", "psfm_destroy", "psfm_n_basis", "psfm_n_spatial",
            "psfm_n_unknowns", "psfm_stamp_dim", "psfm_workspace_bytes", "psfm_stamp_design_floats",
            "psfm_fit_stamps",
            "psfm_solve", "psfm_convolve_image", "psfm_propagate_variance", "psfm_convolve_pair",
            "psfm_subtract", "psfm_match_pair", "psfm_match_pair_static",
            "psfm_status_string", "psfm_batch_workspace_bytes", "psfm_batch_plan",
            "psfm_batch_run", "psfm_batch_run_stage", "psfm_batch_set_tuning", "psfm_batch_graph_capture",
            "psfm_batch_graph_launch", "psfm_batch_destroy", "psfm_wall_clock_hz",
            "psfm_batch_group_capture", "psfm_batch_group_launch", "psfm_batch_group_destroy",
            "psfm_solve_stamps", "psfm_solve_prior", "psfm_cholesky_workspace_bytes",
            "psfm_fit_norm", "psfm_solve_norm", "psfm_quality_eval", "psfm_bin_image",
            "psfm_resample_cov", "psfm_add_images",
            "psfm_dual_workspace_bytes", "psfm_dual_unknowns", "psfm_fit_dual", "psfm_solve_dual",
            "psfm_dual_subtract",
            "psfm_envelope_psf", "psfm_render_workspace_bytes", "psfm_render_target",
            "psfm_stack_reject", "psfm_trace_mask", "psfm_stack_combine",
            "psfm_cholesky_solve", "psfm_cnn_param_count",
            "psfm_cnn_workspace_bytes", "psfm_cnn_forward", "psfm_cnn_loss_grad",
            "psfm_cnn_loss_weights", "psfm_cnn_adam",
            "psfm_cnn_stamp_inputs", "psfm_cnn_targets", "psfm_cnn_local_coeffs",
            "psfm_cnn_standardize", "psfm_cnn_fold_output", "psfm_cnn_excess"]
