"""Matching both images to a common PSF on the GPU (Section 2, Eqs. 1-4 and
the Eq. 9 penalty) against the FP64 oracle, through the C interface.

Tolerances: the stamp sums come from FP32 designs (separable FP32 basis
convolutions of I1 and of I2) folded with FP64 MFMA, so every entry is within
2e-5 of its Cauchy-Schwarz scale sqrt(M_ii M_jj) as in the single form; from
identical stamp sums the solve is FP64 on both sides (kernel sum and chi2/dof
1e-9 relative, coefficients 1e-5 of max|a|, stamp decisions exact); the whole
path meets the single form's targets (kernel sum 1e-4 relative, chi2/dof 1%);
the difference image sums (2h+1)^2 FP32 products per kernel (2e-5 of the
images' scale), its variance 1e-5 relative, masks exact.
"""
import functools
import math

import numpy as np
import pytest

import oracle as O

from gpu_common import hip

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


def render(W, H, xs, ys, fl, sx, sy):
    img = np.zeros((H, W))
    for x0, y0, f in zip(xs, ys, fl):
        r = int(math.ceil(6 * max(sx, sy))) + 1
        xa, xb = max(int(x0) - r, 0), min(int(x0) + r + 1, W)
        ya, yb = max(int(y0) - r, 0), min(int(y0) + r + 1, H)
        if xa >= xb or ya >= yb:
            continue
        y, x = np.mgrid[ya:yb, xa:xb].astype(np.float64)
        img[ya:yb, xa:xb] += f / (2 * math.pi * sx * sy) * np.exp(
            -0.5 * (((x - x0) / sx) ** 2 + ((y - y0) / sy) ** 2))
    return img


def dual_pair(W, H, n_src, n_stamps, R, seed, s1=(1.3, 2.4), s2=(2.4, 1.3)):
    """Two noisy images of the same sources, PSFs elongated along x in I2
    and along y in I1, with a few masked pixels; stamps on sources."""
    rng = np.random.default_rng(seed)
    xs = rng.uniform(5, W - 5, n_src)
    ys = rng.uniform(5, H - 5, n_src)
    fl = np.exp(rng.uniform(math.log(500), math.log(5e4), n_src))
    I1 = render(W, H, xs, ys, fl, *s1) + 30.0
    I2 = render(W, H, xs, ys, fl, *s2) + 45.0
    V1 = (np.abs(I1) + 4.0).astype(np.float32)
    V2 = (np.abs(I2) + 4.0).astype(np.float32)
    I1 = (I1 + np.sqrt(V1) * rng.standard_normal((H, W))).astype(np.float32)
    I2 = (I2 + np.sqrt(V2) * rng.standard_normal((H, W))).astype(np.float32)
    M1 = np.zeros((H, W), np.uint8)
    M2 = np.zeros((H, W), np.uint8)
    M1[rng.integers(0, H, 6), rng.integers(0, W, 6)] = 1
    M2[rng.integers(0, H, 6), rng.integers(0, W, 6)] = 1
    st = [(int(round(x)), int(round(y))) for x, y in zip(xs, ys)]
    st = [p for p in st if R <= p[0] < W - R and R <= p[1] < H - R][:n_stamps]
    st += [(2, 2), (W - 3, H // 2)]                     # off the image: INVALID
    return I1, V1, M1, I2, V2, M2, np.array(st, dtype=np.int32)


CASES = {
    "s0_h8": dict(cfg=dict(h=8, r=12, S=0, P=64), W=320, H=288, n_src=260, n_st=70, seed=1),
    "s1_h10": dict(cfg=dict(h=10, r=14, S=1, P=48), W=333, H=301, n_src=300, n_st=90, seed=2),
}


@functools.lru_cache(maxsize=None)
def _oracle_fit(name):
    c = CASES[name]
    cfg = O.Config(**c["cfg"])
    I1, V1, M1, I2, V2, M2, st = dual_pair(c["W"], c["H"], c["n_src"], c["n_st"], cfg.r + cfg.h, c["seed"])
    return O.fit_dual(cfg, I1, M1, I2, V2, M2, st)


def _setup(name):
    torch, psfm = hip()
    c = CASES[name]
    cfg = O.Config(**c["cfg"])
    ctx = psfm.Context(psfm.Config(**c["cfg"]))
    I1, V1, M1, I2, V2, M2, st = dual_pair(c["W"], c["H"], c["n_src"], c["n_st"],
                                           cfg.r + cfg.h, c["seed"])
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    dev = dict(I1=t(I1), V1=t(V1), M1=t(M1), I2=t(I2), V2=t(V2), M2=t(M2), st=t(st))
    host = dict(I1=I1, V1=V1, M1=M1, I2=I2, V2=V2, M2=M2, st=st, W=c["W"], H=c["H"])
    return torch, psfm, cfg, ctx, dev, host


@pytest.mark.parametrize("name", list(CASES))
def test_fit_dual_parity(name):
    torch, psfm, cfg, ctx, d, h = _setup(name)
    fit = ctx.fit_dual(d["I1"], d["M1"], d["I2"], d["V2"], d["M2"], d["st"])
    ref = _oracle_fit(name)
    assert np.array_equal(_np(fit["flags"]), ref["flags"])
    assert np.array_equal(_np(fit["npix"]), ref["npix"])
    ok = ref["flags"] == 0
    assert ok.sum() >= 20 and (~ok).sum() >= 2
    M, Mr = _np(fit["M"]), ref["M"]
    assert np.all(M[~ok] == 0)
    Md = np.sqrt(np.einsum("sii->si", Mr))
    den = Md[:, :, None] * Md[:, None, :]
    den[den == 0] = 1
    err = np.max(np.abs(M - Mr) / den)
    print(f"{name}: stamp matrix error {err:.2e} of sqrt(M_ii M_jj)")
    assert err < 2e-5
    den_b = Md * np.sqrt(np.maximum(ref["e"], 1e-300))[:, None]
    den_b[den_b == 0] = 1
    assert np.max(np.abs(_np(fit["b"]) - ref["b"]) / den_b) < 2e-5
    assert np.allclose(_np(fit["e"])[ok], ref["e"][ok], rtol=1e-5)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("phi", [0.005, 0.02])
def test_solve_dual_parity_same_sums(name, phi):
    torch, psfm, cfg, ctx, d, h = _setup(name)
    ref_fit = _oracle_fit(name)
    ret, a_ref, chi2_ref, fl_ref, st_ref = O.solve_dual(cfg, h["W"], h["H"], h["st"], ref_fit, phi)
    assert ret == 0
    fit = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in ref_fit.items()}
    sol = ctx.solve_dual(h["W"], h["H"], d["st"], fit, phi)
    st = psfm.read_stats(sol["stats"])
    assert st["info"] == 0 and st["n_iter"] == st_ref["n_iter"] and st["n_used"] == st_ref["n_used"]
    assert np.array_equal(_np(sol["flags"]), fl_ref)
    assert abs(st["kernel_sum_centre"] / st_ref["kernel_sum_centre"] - 1) < 1e-9
    assert abs(st["chi2_dof"] / st_ref["chi2_dof"] - 1) < 1e-9
    a = _np(sol["coeffs"])
    assert a.shape[0] == O.dual_unknowns(cfg) == ctx.N2
    assert np.max(np.abs(a - a_ref)) < 1e-5 * np.max(np.abs(a_ref))
    assert np.allclose(_np(sol["chi2"])[:len(chi2_ref)], chi2_ref, rtol=1e-8, atol=1e-6)


@pytest.mark.parametrize("name", list(CASES))
def test_dual_whole_path(name):
    """GPU fit + solve against the oracle's: the single form's targets; and
    the two-kernel form matches these orthogonally elongated PSFs far better
    than one kernel does."""
    torch, psfm, cfg, ctx, d, h = _setup(name)
    phi = 0.02
    fit = ctx.fit_dual(d["I1"], d["M1"], d["I2"], d["V2"], d["M2"], d["st"])
    sol = ctx.solve_dual(h["W"], h["H"], d["st"], fit, phi)
    st = psfm.read_stats(sol["stats"])
    ref_fit = _oracle_fit(name)
    ret, a_ref, _, fl_ref, st_ref = O.solve_dual(cfg, h["W"], h["H"], h["st"], ref_fit, phi)
    assert st["info"] == 0 and ret == 0
    print(f"{name}: kernel sum {st['kernel_sum_centre']:.6f} vs {st_ref['kernel_sum_centre']:.6f}, "
          f"chi2/dof {st['chi2_dof']:.4f} vs {st_ref['chi2_dof']:.4f}")
    assert abs(st["kernel_sum_centre"] / st_ref["kernel_sum_centre"] - 1) < 1e-4
    assert abs(st["chi2_dof"] / st_ref["chi2_dof"] - 1) < 0.01
    single = ctx.solve(h["W"], h["H"], d["st"], ctx.fit_stamps(d["I1"], d["M1"], d["I2"], d["V2"],
                                                                d["M2"], d["st"]))
    s1 = psfm.read_stats(single["stats"])
    assert s1["info"] == 0 and s1["chi2_dof"] > 2.0 * st["chi2_dof"]


@pytest.mark.parametrize("name", list(CASES))
def test_dual_subtract_parity(name):
    torch, psfm, cfg, ctx, d, h = _setup(name)
    ref_fit = _oracle_fit(name)
    ret, a, _, _, _ = O.solve_dual(cfg, h["W"], h["H"], h["st"], ref_fit, 0.02)
    assert ret == 0
    D, VD, MD = ctx.dual_subtract(torch.from_numpy(a).cuda(), d["I1"], d["V1"], d["M1"], d["I2"],
                                  d["V2"], d["M2"])
    Dr, VDr, MDr = O.dual_apply(cfg, a, h["I1"], h["V1"], h["M1"], h["I2"], h["V2"], h["M2"])
    assert np.array_equal(_np(MD), MDr)
    assert (MDr == O.MASK_CONV_BAD).sum() > 0 and (MDr == O.MASK_CONV_POOR).sum() > 0
    scale = max(np.abs(h["I1"]).max(), np.abs(h["I2"]).max())
    errD = np.abs(_np(D).astype(np.float64) - Dr).max() / scale
    errV = (np.abs(_np(VD).astype(np.float64) - VDr) / np.abs(VDr)).max()
    print(f"{name}: D error {errD:.2e} of max|I|, V_D relative error {errV:.2e}")
    assert errD < 2e-5 and errV < 1e-5


def test_dual_host_checks():
    torch, psfm = hip()
    ctx = psfm.Context(psfm.Config(S=2))          # N2 = 97 * 6 + 1 > 496
    lib = psfm.lib()
    assert lib.psfm_dual_unknowns(ctx.handle) == 583
    n = 4
    L = 2 * ctx.nb
    z = lambda *s, dt=torch.float64: torch.zeros(s, dtype=dt, device="cuda")
    ws = torch.empty(int(lib.psfm_dual_workspace_bytes(ctx.handle, 64, 64, n)), dtype=torch.uint8,
                     device="cuda")
    st = torch.zeros((n, 2), dtype=torch.int32, device="cuda")
    rc = lib.psfm_solve_dual(ctx.handle, 64, 64, st.data_ptr(), n, z(n, L, L).data_ptr(),
                             z(n, L).data_ptr(), z(n).data_ptr(), z(n, dt=torch.int32).data_ptr(),
                             z(n, dt=torch.int32).data_ptr(), 0.01, z(583).data_ptr(), z(n).data_ptr(),
                             torch.zeros(psfm.STATS_BYTES, dtype=torch.uint8, device="cuda").data_ptr(),
                             ws.data_ptr(), ws.numel(), None)
    assert rc == -7                               # PSFM_ERR_UNSUPPORTED
    assert lib.psfm_solve_dual(ctx.handle, 64, 64, None, 0, None, None, None, None, None, -1.0,
                               None, None, None, None, 0, None) == -1
