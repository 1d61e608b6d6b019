"""ctypes front end of the FP64 oracle (``psfm_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke`` and
the CPU-baseline leg of ``bench.py``; never by the product path.  The arithmetic
lives in the C file; this module only marshals numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "psfm_oracle.c")
_LIB = os.path.join(_HERE, "libpsfm_oracle.so")

MAX_GAUSS = 8
STAMP_INVALID, STAMP_REJECTED, STAMP_NONFINITE = 1, 2, 4
MASK_BAD, MASK_CONV_BAD, MASK_CONV_POOR = 1, 2, 4


STAMP_RESERVE = 32
CUT_FEW_STAMPS, CUT_MEAN_DEV, CUT_RMS_DEV, CUT_MOMENT1, CUT_MOMENT2, CUT_DECONV = 1, 2, 4, 8, 16, 32


class OrcQuality(C.Structure):
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


class OrcConfig(C.Structure):
    _fields_ = [
        ("n_gauss", C.c_int),
        ("sigma", C.c_double * MAX_GAUSS),
        ("degree", C.c_int * MAX_GAUSS),
        ("h", C.c_int),
        ("S", C.c_int),
        ("r", C.c_int),
        ("P", C.c_int),
        ("clip_sigma", C.c_double),
        ("max_iter", C.c_int),
        ("min_stamps", C.c_int),
        ("bad_frac", C.c_double),
    ]


class OrcStats(C.Structure):
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
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-Wall", "-Wno-unused-function", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        P = C.c_void_p
        i, i64, d = C.c_int, C.c_int64, C.c_double
        cfgp = C.POINTER(OrcConfig)
        sig = {
            "orc_n_basis": (i, [cfgp]),
            "orc_n_spatial": (i, [cfgp]),
            "orc_n_unknowns": (i, [cfgp]),
            "orc_n_patches": (i, [cfgp, i, i]),
            "orc_basis": (None, [cfgp, P]),
            "orc_spatial": (None, [i, d, d, i, i, P]),
            "orc_local_coeffs": (None, [cfgp, P, d, d, i, i, P]),
            "orc_kernel_at": (None, [cfgp, P, P, d, d, i, i, P]),
            "orc_fit_stamps": (None, [cfgp, P, P, P, P, P, P, i, i, i64, P, i, P, P, P, P, P, P]),
            "orc_assemble": (None, [cfgp, i, i, P, i, P, P, P, P, P]),
            "orc_cholesky_solve": (i, [i, P, P, P]),
            "orc_stamp_chi2": (d, [cfgp, P, i, i, i, i, P, P, d]),
            "orc_solve": (i, [cfgp, i, i, P, i, P, P, P, P, P, P, P, C.POINTER(OrcStats)]),
            "orc_bad_radius": (i, [P, i, d]),
            "orc_cov_raw": (None, [P, i, P, i, P]),
            "orc_cov_factor": (d, [P, i, P, i]),
            "orc_patch_kernel": (None, [cfgp, P, P, i, i, i, P]),
            "orc_convolve_image": (None, [cfgp, P, P, P, P, i, i, i64, P, P]),
            "orc_propagate_variance": (None, [cfgp, P, P, P, P, i, i, i64, P, i, P, P, i, P]),
            "orc_subtract": (None, [cfgp, P, P, P, P, P, P, P, i, i, i64, P, i, P, i, P, P, P, P,
                                    i]),
            "orc_convolve_region": (None, [cfgp, P, P, P, P, P, i, i, i64, P, i, i, i, i, i, P, P,
                                           P]),
            "orc_fit_norm": (None, [cfgp, P, P, P, i, i, i64, P, i, P, P]),
            "orc_norm_solve": (i, [i, P, P, P, P]),
            "orc_solve_norm": (i, [cfgp, i, i, P, i, P, P, P, P, P, P, P, P, P,
                                   C.POINTER(OrcStats), C.POINTER(C.c_int)]),
            "orc_quality_eval": (None, [cfgp, P, P, P, P, P, i, i, i64, P, i, P, d, P,
                                        C.POINTER(OrcQuality)]),
            "orc_bin": (None, [P, P, P, i, i, i64, i, P, i, P, P, P, P, i, P]),
            "orc_resample_cov": (None, [P, i, d, P, i]),
            "orc_add_images": (None, [d, P, P, P, P, i, d, P, P, P, P, i, i, i, i64, P, P, P, P, i]),
            "orc_envelope_psf": (d, [P, i, i, P]),
            "orc_render_target": (None, [P, i, d, i, i, i64, P]),
            "orc_stack_reject": (None, [i, P, P, P, i64, i, i, i64, d, P]),
            "orc_trace_mask": (None, [cfgp, P, P, P, i, i, i64, d, P]),
            "orc_stack_combine": (None, [i, P, P, P, i64, i, i, i64, P, i, P, P, P, P, P]),
            "orc_dual_unknowns": (i, [cfgp]),
            "orc_fit_dual": (None, [cfgp, P, P, P, P, P, P, i, i, i64, P, i, P, P, P, P, P, P]),
            "orc_penalty_q": (None, [cfgp, P, P]),
            "orc_solve_dual": (i, [cfgp, P, i, i, P, i, P, P, P, P, P, d, P, P, C.POINTER(OrcStats)]),
            "orc_dual_kernels": (None, [cfgp, P, P, d, d, i, i, P, P]),
            "orc_dual_apply": (None, [cfgp, P, P, P, P, P, P, P, P, i, i, i64, P, P, P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(_lib, name)
            fn.restype = res
            fn.argtypes = args
    return _lib


def set_threads(n: int) -> None:
    """Number of OpenMP threads the oracle's parallel loops use from now on
    (the OpenMP runtime the library is linked against)."""
    lib().omp_set_num_threads(C.c_int(int(n)))


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


@dataclasses.dataclass
class Config:
    """Method parameters (the same fields as the C interface's config)."""
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

    @classmethod
    def from_workload(cls, wl, **kw):
        base = dict(sigmas=tuple(wl.sigmas), degrees=tuple(wl.degrees), h=wl.kernel_half,
                    S=wl.spatial_order, r=wl.stamp_half, P=wl.patch)
        base.update(kw)
        return cls(**base)

    def c(self) -> OrcConfig:
        cfg = OrcConfig()
        cfg.n_gauss = len(self.sigmas)
        for j, (s, dg) in enumerate(zip(self.sigmas, self.degrees)):
            cfg.sigma[j] = s
            cfg.degree[j] = dg
        cfg.h, cfg.S, cfg.r, cfg.P = self.h, self.S, self.r, self.P
        cfg.clip_sigma, cfg.max_iter, cfg.min_stamps = self.clip_sigma, self.max_iter, self.min_stamps
        cfg.bad_frac = self.bad_frac
        return cfg

    @property
    def n_basis(self):
        return sum((d + 1) * (d + 2) // 2 for d in self.degrees)

    @property
    def n_spatial(self):
        return (self.S + 1) * (self.S + 2) // 2

    @property
    def n_unknowns(self):
        return self.n_basis * self.n_spatial + 1

    @property
    def taps(self):
        return (2 * self.h + 1) ** 2


def basis(cfg: Config) -> np.ndarray:
    """[n_basis, 2h+1, 2h+1] float64 kernel basis."""
    K = 2 * cfg.h + 1
    out = np.zeros((cfg.n_basis, K, K), dtype=np.float64)
    lib().orc_basis(C.byref(cfg.c()), _p(out))
    return out


def spatial(cfg: Config, x: float, y: float, W: int, H: int) -> np.ndarray:
    g = np.zeros(cfg.n_spatial, dtype=np.float64)
    lib().orc_spatial(cfg.S, float(x), float(y), W, H, _p(g))
    return g


def local_coeffs(cfg: Config, a: np.ndarray, x: float, y: float, W: int, H: int) -> np.ndarray:
    a = _c(a, np.float64)
    out = np.zeros(cfg.n_basis + 1, dtype=np.float64)
    lib().orc_local_coeffs(C.byref(cfg.c()), _p(a), float(x), float(y), W, H, _p(out))
    return out


def kernel_at(cfg: Config, a: np.ndarray, x: float, y: float, W: int, H: int,
              kb: Optional[np.ndarray] = None) -> np.ndarray:
    kb = basis(cfg) if kb is None else kb
    a = _c(a, np.float64)
    K = np.zeros((2 * cfg.h + 1, 2 * cfg.h + 1), dtype=np.float64)
    lib().orc_kernel_at(C.byref(cfg.c()), _p(kb), _p(a), float(x), float(y), W, H, _p(K))
    return K


def fit_stamps(cfg: Config, I1, M1, I2, V2, M2, stamps, kb=None, V1=None):
    """Per-stamp sums: returns dict(M [n,L,L], b [n,L], e [n], npix [n], flags [n]).
    With V1 the weights are 1 / (V1 + V2), else 1 / V2."""
    kb = basis(cfg) if kb is None else kb
    I1, I2, V2 = (_c(a, np.float32) for a in (I1, I2, V2))
    V1 = None if V1 is None else _c(V1, np.float32)
    M1, M2 = _c(M1, np.uint8), _c(M2, np.uint8)
    H, W = I1.shape
    xy = _c(stamps, np.int32).reshape(-1, 2)
    n = xy.shape[0]
    L = cfg.n_basis + 1
    Ms = np.zeros((n, L, L)); bs = np.zeros((n, L)); es = np.zeros(n)
    npix = np.zeros(n, dtype=np.int32); flags = np.zeros(n, dtype=np.int32)
    lib().orc_fit_stamps(C.byref(cfg.c()), _p(kb), _p(I1), _p(M1), _p(I2), _p(V2), _p(M2), W, H,
                         W, _p(xy), n, _p(Ms), _p(bs), _p(es), _p(npix), _p(flags), _p(V1))
    return dict(M=Ms, b=bs, e=es, npix=npix, flags=flags)


def assemble(cfg: Config, W, H, stamps, Ms, bs, used):
    N = cfg.n_unknowns
    M = np.zeros((N, N)); b = np.zeros(N)
    xy = _c(stamps, np.int32).reshape(-1, 2)
    lib().orc_assemble(C.byref(cfg.c()), W, H, _p(xy), xy.shape[0], _p(_c(Ms, np.float64)),
                       _p(_c(bs, np.float64)), _p(_c(used, np.uint8)), _p(M), _p(b))
    return M, b


def cholesky_solve(M, b):
    M = _c(M, np.float64); b = _c(b, np.float64)
    x = np.zeros_like(b)
    info = lib().orc_cholesky_solve(M.shape[0], _p(M), _p(b), _p(x))
    return x, info


def stamp_chi2(cfg: Config, a, W, H, x, y, Ms, bs, es) -> float:
    return lib().orc_stamp_chi2(C.byref(cfg.c()), _p(_c(a, np.float64)), W, H, int(x), int(y),
                                _p(_c(Ms, np.float64)), _p(_c(bs, np.float64)), float(es))


def solve(cfg: Config, W, H, stamps, fit, flags=None):
    """Solution with rejection.  Returns (ret, coeffs, chi2 [n], flags [n], stats dict)."""
    xy = _c(stamps, np.int32).reshape(-1, 2)
    n = xy.shape[0]
    fl = _c(fit["flags"] if flags is None else flags, np.int32).copy()
    a = np.zeros(cfg.n_unknowns); chi2 = np.zeros(n)
    st = OrcStats()
    ret = lib().orc_solve(C.byref(cfg.c()), W, H, _p(xy), n, _p(_c(fit["M"], np.float64)),
                          _p(_c(fit["b"], np.float64)), _p(_c(fit["e"], np.float64)),
                          _p(_c(fit["npix"], np.int32)), _p(fl), _p(a), _p(chi2), C.byref(st))
    return ret, a, chi2, fl, st.as_dict()


def bad_radius(K, h, frac=0.2) -> int:
    return lib().orc_bad_radius(_p(_c(K, np.float64)), h, frac)


def cov_raw(K, h, cov_in=None, c_in=0):
    R = 2 * h + c_in
    out = np.zeros((2 * R + 1, 2 * R + 1))
    lib().orc_cov_raw(_p(_c(K, np.float64)), h, _p(None if cov_in is None else _c(cov_in, np.float64)),
                      c_in, _p(out))
    return out


def cov_factor(K, h, cov_in=None, c_in=0) -> float:
    return lib().orc_cov_factor(_p(_c(K, np.float64)), h,
                                _p(None if cov_in is None else _c(cov_in, np.float64)), c_in)


def patch_kernel(cfg: Config, a, W, H, p, kb=None):
    kb = basis(cfg) if kb is None else kb
    K = np.zeros((2 * cfg.h + 1, 2 * cfg.h + 1))
    lib().orc_patch_kernel(C.byref(cfg.c()), _p(kb), _p(_c(a, np.float64)), W, H, p, _p(K))
    return K


def n_patches(cfg: Config, W, H) -> int:
    return lib().orc_n_patches(C.byref(cfg.c()), W, H)


def convolve_image(cfg: Config, a, I, M, kb=None):
    kb = basis(cfg) if kb is None else kb
    I = _c(I, np.float32); M = _c(M, np.uint8)
    H, W = I.shape
    out = np.zeros((H, W), dtype=np.float32); om = np.zeros((H, W), dtype=np.uint8)
    lib().orc_convolve_image(C.byref(cfg.c()), _p(kb), _p(_c(a, np.float64)), _p(I), _p(M), W, H,
                             W, _p(out), _p(om))
    return out, om


def propagate_variance(cfg: Config, a, V, M, cov_in=None, c_in=0, c_out=10, kb=None):
    kb = basis(cfg) if kb is None else kb
    V = _c(V, np.float32); M = _c(M, np.uint8)
    H, W = V.shape
    out = np.zeros((H, W), dtype=np.float32)
    cov = np.zeros((2 * c_out + 1, 2 * c_out + 1))
    disc = C.c_double(0.0)
    lib().orc_propagate_variance(C.byref(cfg.c()), _p(kb), _p(_c(a, np.float64)), _p(V), _p(M), W,
                                 H, W, _p(None if cov_in is None else _c(cov_in, np.float64)), c_in,
                                 _p(out), _p(cov), c_out, C.byref(disc))
    return out, cov, disc.value


def convolve_region(cfg: Config, a, I, V, M, rect, cov_in=None, c_in=0, kb=None):
    """Image and variance convolution restricted to rect = (x0, y0, x1, y1) of
    the full image; returns (conv, mask, var) of the rectangle's shape."""
    kb = basis(cfg) if kb is None else kb
    M = _c(M, np.uint8)
    H, W = M.shape
    x0, y0, x1, y1 = rect
    Ic = None if I is None else _c(I, np.float32)
    Vc = None if V is None else _c(V, np.float32)
    out = np.zeros((y1 - y0, x1 - x0), np.float32) if I is not None else None
    om = np.zeros((y1 - y0, x1 - x0), np.uint8) if I is not None else None
    var = np.zeros((y1 - y0, x1 - x0), np.float32) if V is not None else None
    lib().orc_convolve_region(C.byref(cfg.c()), _p(kb), _p(_c(a, np.float64)), _p(Ic), _p(Vc),
                              _p(M), W, H, W,
                              _p(None if cov_in is None else _c(cov_in, np.float64)), c_in,
                              x0, y0, x1, y1, _p(out), _p(om), _p(var))
    return out, om, var


def subtract(cfg: Config, a, I2, V2, M2, conv, conv_var, conv_mask, cov_conv, cov2=None, c_d=None):
    I2, V2, conv, conv_var = (_c(x, np.float32) for x in (I2, V2, conv, conv_var))
    M2, conv_mask = _c(M2, np.uint8), _c(conv_mask, np.uint8)
    cov_conv = _c(cov_conv, np.float64)
    cc = (cov_conv.shape[0] - 1) // 2
    c2 = 0 if cov2 is None else (np.asarray(cov2).shape[0] - 1) // 2
    cd = max(cc, c2) if c_d is None else c_d
    H, W = I2.shape
    D = np.zeros((H, W), np.float32); VD = np.zeros((H, W), np.float32)
    MD = np.zeros((H, W), np.uint8); CD = np.zeros((2 * cd + 1, 2 * cd + 1))
    lib().orc_subtract(C.byref(cfg.c()), _p(_c(a, np.float64)), _p(I2), _p(V2), _p(M2), _p(conv),
                       _p(conv_var), _p(conv_mask), W, H, W,
                       _p(None if cov2 is None else _c(cov2, np.float64)), c2, _p(cov_conv), cc,
                       _p(D), _p(VD), _p(MD), _p(CD), cd)
    return D, VD, MD, CD


def match_pair(cfg: Config, pair, c_out: int = 10):
    """The whole path on one pair: fit -> solve -> convolve -> variance -> subtract."""
    kb = basis(cfg)
    fit = fit_stamps(cfg, pair.I1, pair.M1, pair.I2, pair.V2, pair.M2, pair.stamps, kb=kb)
    W, H = pair.width, pair.height
    ret, a, chi2, flags, st = solve(cfg, W, H, pair.stamps, fit)
    out = dict(fit=fit, ret=ret, coeffs=a, chi2=chi2, flags=flags, stats=st)
    if ret != 0:
        return out
    conv, cmask = convolve_image(cfg, a, pair.I1, pair.M1, kb=kb)
    var, cov, disc = propagate_variance(cfg, a, pair.V1, pair.M1, c_out=c_out, kb=kb)
    D, VD, MD, CD = subtract(cfg, a, pair.I2, pair.V2, pair.M2, conv, var, cmask, cov)
    out.update(conv=conv, conv_mask=cmask, var=var, cov=cov, cov_discarded=disc, diff=D,
               diff_var=VD, diff_mask=MD, cov_diff=CD)
    return out


# ---------------------------------------------------------------- the paper's
# normalisation and quality mode (Sections 3.2, 3.3, 3.6, 3.7)

def fit_norm(cfg: Config, I1, I2, stamps, flags, kb=None):
    """Per-stamp unweighted sums [n, 5]: npix, sum A0, sum I2, sum A0^2, sum A0 I2."""
    kb = basis(cfg) if kb is None else kb
    I1, I2 = _c(I1, np.float32), _c(I2, np.float32)
    H, W = I1.shape
    xy = _c(stamps, np.int32).reshape(-1, 2)
    n = xy.shape[0]
    out = np.zeros((n, 5))
    lib().orc_fit_norm(C.byref(cfg.c()), _p(kb), _p(I1), _p(I2), W, H, W, _p(xy), n,
                       _p(_c(flags, np.int32)), _p(out))
    return out


def norm_solve(norm, used):
    """(ret, b0, d0) from the stamp totals of the stamps in use."""
    norm = _c(norm, np.float64)
    b0, d0 = C.c_double(0.0), C.c_double(0.0)
    ret = lib().orc_norm_solve(norm.shape[0], _p(norm), _p(_c(used, np.uint8)), C.byref(b0),
                               C.byref(d0))
    return ret, b0.value, d0.value


def solve_norm(cfg: Config, W, H, stamps, fit, norm, flags=None, group=None):
    """Paper's normalisation mode.  Returns (ret, coeffs, chi2, flags, stats, n_replaced)."""
    xy = _c(stamps, np.int32).reshape(-1, 2)
    n = xy.shape[0]
    fl = _c(fit["flags"] if flags is None else flags, np.int32).copy()
    a = np.zeros(cfg.n_unknowns); chi2 = np.zeros(n)
    st = OrcStats()
    nrep = C.c_int(0)
    ret = lib().orc_solve_norm(C.byref(cfg.c()), W, H, _p(xy), n, _p(_c(fit["M"], np.float64)),
                               _p(_c(fit["b"], np.float64)), _p(_c(fit["e"], np.float64)),
                               _p(_c(fit["npix"], np.int32)), _p(_c(norm, np.float64)),
                               _p(None if group is None else _c(group, np.int32)), _p(fl), _p(a),
                               _p(chi2), C.byref(st), C.byref(nrep))
    return ret, a, chi2, fl, st.as_dict(), nrep.value


def quality(cfg: Config, a, I1, I2, V2, stamps, flags, soft=0.0, kb=None):
    """Quality record and per-stamp deviations of a solution (Section 3.6)."""
    kb = basis(cfg) if kb is None else kb
    I1, I2, V2 = (_c(x, np.float32) for x in (I1, I2, V2))
    H, W = I1.shape
    xy = _c(stamps, np.int32).reshape(-1, 2)
    n = xy.shape[0]
    dev = np.zeros(n)
    q = OrcQuality()
    lib().orc_quality_eval(C.byref(cfg.c()), _p(kb), _p(_c(a, np.float64)), _p(I1), _p(I2), _p(V2), W,
                           H, W, _p(xy), n, _p(_c(flags, np.int32)), float(soft), _p(dev), C.byref(q))
    return q.as_dict(), dev


# ------------------------------------------------ noise-model operations
# beyond convolution (Section 4.3)

def bin_image(I, V, M, B, cov_in=None, c_out=4):
    """Integer binning: (Ib, Vb, Mb, cov_b, discarded)."""
    I, V = _c(I, np.float32), _c(V, np.float32)
    M = _c(M, np.uint8)
    H, W = I.shape
    Wb, Hb = W // B, H // B
    Ib = np.zeros((Hb, Wb), np.float32); Vb = np.zeros((Hb, Wb), np.float32)
    Mb = np.zeros((Hb, Wb), np.uint8); cov = np.zeros((2 * c_out + 1, 2 * c_out + 1))
    c_in = 0 if cov_in is None else (np.asarray(cov_in).shape[0] - 1) // 2
    disc = C.c_double(0.0)
    lib().orc_bin(_p(I), _p(V), _p(M), W, H, W, B,
                  _p(None if cov_in is None else _c(cov_in, np.float64)), c_in, _p(Ib), _p(Vb), _p(Mb),
                  _p(cov), c_out, C.byref(disc))
    return Ib, Vb, Mb, cov, disc.value


def resample_cov(cov_in, scale, c_out):
    cov_in = _c(cov_in, np.float64)
    out = np.zeros((2 * c_out + 1, 2 * c_out + 1))
    lib().orc_resample_cov(_p(cov_in), (cov_in.shape[0] - 1) // 2, float(scale), _p(out), c_out)
    return out


def add_images(alpha, Ia, Va, Ma, Ca, beta, Ib, Vb, Mb, Cb, cs):
    """S = alpha Ia + beta Ib with variance, mask and pseudo-matrix."""
    Ia, Va, Ib, Vb = (_c(x, np.float32) for x in (Ia, Va, Ib, Vb))
    Ma, Mb = _c(Ma, np.uint8), _c(Mb, np.uint8)
    H, W = Ia.shape
    S = np.zeros((H, W), np.float32); VS = np.zeros((H, W), np.float32)
    MS = np.zeros((H, W), np.uint8); CS = np.zeros((2 * cs + 1, 2 * cs + 1))
    ca = 0 if Ca is None else (np.asarray(Ca).shape[0] - 1) // 2
    cb = 0 if Cb is None else (np.asarray(Cb).shape[0] - 1) // 2
    lib().orc_add_images(float(alpha), _p(Ia), _p(Va), _p(Ma),
                         _p(None if Ca is None else _c(Ca, np.float64)), ca, float(beta), _p(Ib), _p(Vb),
                         _p(Mb), _p(None if Cb is None else _c(Cb, np.float64)), cb, W, H, W, _p(S),
                         _p(VS), _p(MS), _p(CS), cs)
    return S, VS, MS, CS


# ---------------------------------------------- PSF homogenisation (Section 5)

def envelope_psf(params, half):
    """(sigma_env, envelope image) from n x 3 (sigma_major, sigma_minor, angle)."""
    params = _c(params, np.float64).reshape(-1, 3)
    env = np.zeros((2 * half + 1, 2 * half + 1))
    s = lib().orc_envelope_psf(_p(params), params.shape[0], half, _p(env))
    return s, env


def render_target(src, sigma, W, H):
    src = _c(src, np.float64).reshape(-1, 3)
    out = np.zeros((H, W), np.float32)
    lib().orc_render_target(_p(src), src.shape[0], float(sigma), W, H, W, _p(out))
    return out


def stack_reject(I, V, M, nsigma):
    """I, V, M: [n, H, W]; returns outlier flags [n, H, W] (uint8)."""
    I, V = _c(I, np.float32), _c(V, np.float32)
    M = _c(M, np.uint8)
    n, H, W = I.shape
    out = np.zeros((n, H, W), np.uint8)
    lib().orc_stack_reject(n, _p(I), _p(V), _p(M), H * W, W, H, W, float(nsigma), _p(out))
    return out


def trace_mask(cfg: Config, a, outl, frac, kb=None):
    kb = basis(cfg) if kb is None else kb
    outl = _c(outl, np.uint8)
    H, W = outl.shape
    bad = np.zeros((H, W), np.uint8)
    lib().orc_trace_mask(C.byref(cfg.c()), _p(kb), _p(_c(a, np.float64)), _p(outl), W, H, W,
                         float(frac), _p(bad))
    return bad


def stack_combine(I, V, M, covs):
    """I, V, M: [n, H, W]; covs [n, Cw, Cw].  Returns (S, VS, MS, CS, weights)."""
    I, V = _c(I, np.float32), _c(V, np.float32)
    M = _c(M, np.uint8)
    covs = _c(covs, np.float64)
    n, H, W = I.shape
    ck = (covs.shape[1] - 1) // 2
    S = np.zeros((H, W), np.float32); VS = np.zeros((H, W), np.float32)
    MS = np.zeros((H, W), np.uint8); CS = np.zeros((2 * ck + 1, 2 * ck + 1)); w = np.zeros(n)
    lib().orc_stack_combine(n, _p(I), _p(V), _p(M), H * W, W, H, W, _p(covs), ck, _p(S), _p(VS),
                            _p(MS), _p(CS), _p(w))
    return S, VS, MS, CS, w


# ---------------------------------------------------------------- two kernels

def dual_unknowns(cfg: Config) -> int:
    return (2 * cfg.n_basis - 1) * cfg.n_spatial + 1


def fit_dual(cfg: Config, I1, M1, I2, V2, M2, stamps, kb=None, V1=None):
    """Per-stamp sums of the two-kernel form: dict(M [n,L2,L2], b [n,L2], e, npix, flags), L2 = 2 nb.
    With V1 the weights are 1 / (V1 + V2), else 1 / V2."""
    kb = basis(cfg) if kb is None else kb
    I1, I2, V2 = (_c(a, np.float32) for a in (I1, I2, V2))
    V1 = None if V1 is None else _c(V1, np.float32)
    M1, M2 = _c(M1, np.uint8), _c(M2, np.uint8)
    H, W = I1.shape
    xy = _c(stamps, np.int32).reshape(-1, 2)
    n = xy.shape[0]
    L = 2 * cfg.n_basis
    Ms = np.zeros((n, L, L)); bs = np.zeros((n, L)); es = np.zeros(n)
    npix = np.zeros(n, dtype=np.int32); flags = np.zeros(n, dtype=np.int32)
    lib().orc_fit_dual(C.byref(cfg.c()), _p(kb), _p(I1), _p(M1), _p(I2), _p(V2), _p(M2), W, H, W,
                       _p(xy), n, _p(Ms), _p(bs), _p(es), _p(npix), _p(flags), _p(V1))
    return dict(M=Ms, b=bs, e=es, npix=npix, flags=flags)


def penalty_q(cfg: Config, kb=None) -> np.ndarray:
    kb = basis(cfg) if kb is None else kb
    Q = np.zeros(cfg.n_basis)
    lib().orc_penalty_q(C.byref(cfg.c()), _p(kb), _p(Q))
    return Q


def solve_dual(cfg: Config, W, H, stamps, fit, phi, flags=None, kb=None):
    """Two-kernel solution with rejection.  Returns (ret, coeffs, chi2, flags, stats)."""
    kb = basis(cfg) if kb is None else kb
    xy = _c(stamps, np.int32).reshape(-1, 2)
    n = xy.shape[0]
    fl = _c(fit["flags"] if flags is None else flags, np.int32).copy()
    a = np.zeros(dual_unknowns(cfg)); chi2 = np.zeros(n)
    st = OrcStats()
    ret = lib().orc_solve_dual(C.byref(cfg.c()), _p(kb), W, H, _p(xy), n, _p(_c(fit["M"], np.float64)),
                               _p(_c(fit["b"], np.float64)), _p(_c(fit["e"], np.float64)),
                               _p(_c(fit["npix"], np.int32)), _p(fl), float(phi), _p(a), _p(chi2),
                               C.byref(st))
    return ret, a, chi2, fl, st.as_dict()


def dual_kernels(cfg: Config, a, x, y, W, H, kb=None):
    kb = basis(cfg) if kb is None else kb
    K = 2 * cfg.h + 1
    K1 = np.zeros((K, K)); K2 = np.zeros((K, K))
    lib().orc_dual_kernels(C.byref(cfg.c()), _p(kb), _p(_c(a, np.float64)), float(x), float(y), W, H,
                           _p(K1), _p(K2))
    return K1, K2


def dual_apply(cfg: Config, a, I1, V1, M1, I2, V2, M2, kb=None):
    """(D, V_D, mask_D) of the two-kernel form."""
    kb = basis(cfg) if kb is None else kb
    I1, V1, I2, V2 = (_c(x, np.float32) for x in (I1, V1, I2, V2))
    M1, M2 = _c(M1, np.uint8), _c(M2, np.uint8)
    H, W = I1.shape
    D = np.zeros((H, W), np.float32); VD = np.zeros((H, W), np.float32); MD = np.zeros((H, W), np.uint8)
    lib().orc_dual_apply(C.byref(cfg.c()), _p(kb), _p(_c(a, np.float64)), _p(I1), _p(V1), _p(M1), _p(I2),
                         _p(V2), _p(M2), W, H, W, _p(D), _p(VD), _p(MD))
    return D, VD, MD
