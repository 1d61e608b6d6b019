"""psfm_match_pair_static (the entry point for callers that cannot allocate):
through the C interface it gives psfm_match_pair's outputs bit for bit, on
two calls in a row with the second on a smaller image (the static scratch
keeps the first call's contents), and rejects an image whose scratch would
not fit the static array before launching anything."""
import gc

import numpy as np
import pytest

from paper_1901_09999_amd import synth

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


def _corr(rng, c):
    import torch
    q = rng.uniform(0.0, 1.0, (2 * c + 1, 2 * c + 1))
    m = np.array([[np.sum(q[max(0, -dy):q.shape[0] - max(0, dy), max(0, -dx):q.shape[1] - max(0, dx)] *
                          q[max(0, dy):q.shape[0] - max(0, -dy), max(0, dx):q.shape[1] - max(0, -dx)])
                   for dx in range(-c, c + 1)] for dy in range(-c, c + 1)])
    return torch.from_numpy(m / m[c, c]).cuda()


def _case(psfm, torch, W, H, h, P, seed, c_in):
    base = synth.WORKLOADS["pair2048"]
    wl = synth.scaled(base, f"na{W}x{H}", W, H, n_sources=max(40, W * H // 600), n_stamps=30,
                      kernel_half=h, patch=P)
    pair = synth.make_pair(wl, seed)
    ctx = psfm.Context(psfm.Config.from_workload(wl))
    d = psfm.to_device(pair)
    rng = np.random.default_rng(seed)
    a = np.zeros(ctx.N)
    a[0] = 1.0
    a[:-1] += 0.02 * rng.standard_normal(ctx.N - 1)
    a[-1] = 1.5
    at = torch.from_numpy(a).cuda()
    cin = _corr(rng, c_in) if c_in else None
    c2 = _corr(rng, c_in + 1) if c_in else None
    return ctx, d, at, cin, c2


def _outputs(torch, ref_like_I, ref_like_M, c_out, cd):
    return dict(diff=torch.empty_like(ref_like_I), diff_var=torch.empty_like(ref_like_I),
                diff_mask=torch.empty_like(ref_like_M),
                cov_diff=torch.empty((2 * cd + 1,) * 2, dtype=torch.float64, device="cuda"))


def test_static_entry_matches_workspace_entry():
    import torch
    from paper_1901_09999_amd import psfm
    assert torch.cuda.is_available()
    # first call on a large image, second on a smaller ragged one
    for (W, H, h, P, seed, c_in) in [(1536, 1280, 10, 64, 41, 1), (300, 217, 5, 50, 42, 2)]:
        print(f"no-alloc case {W}x{H} h={h} P={P} c_in={c_in}", flush=True)
        ctx, d, at, cin, c2 = _case(psfm, torch, W, H, h, P, seed, c_in)
        c_out = 2 * h + 2
        cd = max(c_out, c_in + 1)
        s_ws = torch.zeros(psfm.STATS_BYTES, dtype=torch.uint8, device="cuda")
        s_st = torch.zeros(psfm.STATS_BYTES, dtype=torch.uint8, device="cuda")
        conv_w = torch.empty_like(d["I1"]); cm_w = torch.empty_like(d["M1"])
        var_w = torch.empty_like(d["V1"])
        conv_s = torch.full_like(d["I1"], -7.0); cm_s = torch.full_like(d["M1"], 9)
        var_s = torch.full_like(d["V1"], -7.0)
        cov_w = torch.empty((2 * c_out + 1,) * 2, dtype=torch.float64, device="cuda")
        cov_s = torch.full_like(cov_w, -7.0)
        out_w = _outputs(torch, d["I2"], d["M2"], c_out, cd)
        out_s = _outputs(torch, d["I2"], d["M2"], c_out, cd)
        for v in out_s.values():
            v.fill_(3)
        ref = ctx.match(at, d["I1"], d["V1"], d["M1"], d["I2"], d["V2"], d["M2"], cov1=cin,
                        cov2=c2, c_out=c_out, c_d=cd, stats=s_ws, out=out_w, cov_conv=cov_w,
                        conv=conv_w, conv_mask=cm_w, conv_var=var_w)
        torch.cuda.synchronize()
        gc.collect()
        before = torch.cuda.memory_allocated()
        got = ctx.match_static(at, d["I1"], d["V1"], d["M1"], d["I2"], d["V2"], d["M2"], cov1=cin,
                               cov2=c2, c_out=c_out, c_d=cd, stats=s_st, out=out_s,
                               cov_conv=cov_s, conv=conv_s, conv_mask=cm_s, conv_var=var_s)
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() <= before     # nothing allocated by the call
        for k in ("diff", "diff_var", "diff_mask", "cov_diff", "cov"):
            assert np.array_equal(_np(got[k]), _np(ref[k])), k
        assert np.array_equal(_np(conv_s), _np(conv_w))
        assert np.array_equal(_np(cm_s), _np(cm_w))
        assert np.array_equal(_np(var_s), _np(var_w))
        assert psfm.read_stats(s_st)["cov_discarded_frac"] == \
            psfm.read_stats(s_ws)["cov_discarded_frac"]
        # the pair itself was matched: unflagged difference pixels are finite
        dm = _np(got["diff_mask"])
        assert np.isfinite(_np(got["diff"])[dm == 0]).all() and (dm == 0).mean() > 0.5


def test_static_entry_rejects_oversized_images():
    """8-px patches on a 4096^2 image need 262144 tiles x 32 bytes of variance
    sums: more than the static array holds; the call returns
    PSFM_ERR_WORKSPACE before launching (the buffers are real, full-size
    allocations all the same)."""
    import torch
    from paper_1901_09999_amd import psfm
    W = H = 4096
    ctx = psfm.Context(psfm.Config(h=3, P=8, r=6))
    f = torch.zeros((H, W), dtype=torch.float32, device="cuda")
    m = torch.zeros((H, W), dtype=torch.uint8, device="cuda")
    a = torch.zeros(ctx.N, dtype=torch.float64, device="cuda")
    a[0] = 1.0
    with pytest.raises(psfm.PsfmError, match="workspace"):
        ctx.match_static(a, f, f, m, f, f, m, c_out=6)
    # the same image with 64-px patches fits
    ctx64 = psfm.Context(psfm.Config(h=3, P=64, r=6))
    r = ctx64.match_static(a, f, f + 1.0, m, f, f + 1.0, m, c_out=6)
    torch.cuda.synchronize()
    assert float(r["diff"].abs().max()) == 0.0 and float(r["diff_var"].min()) > 1.0
