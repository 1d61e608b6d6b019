"""Shared helpers of the GPU parity tests: run the HIP path (through the C
interface) and the FP64 oracle on the same seeded inputs."""
import functools

import numpy as np

import oracle as O
from paper_1901_09999_amd import synth


def hip():
    import torch
    from paper_1901_09999_amd import psfm

    assert torch.cuda.is_available(), "a HIP device is required"
    return torch, psfm


@functools.lru_cache(maxsize=8)
def pair_for(name: str, seed: int, width: int = 0, height: int = 0, n_stamps: int = 0, **kw):
    wl = synth.WORKLOADS[name]
    if width:
        wl = synth.scaled(wl, f"{name}_{width}x{height}", width, height,
                          n_stamps=n_stamps or wl.n_stamps, **kw)
    return wl, synth.make_pair(wl, seed)


@functools.lru_cache(maxsize=8)
def oracle_run(name: str, seed: int, width: int = 0, height: int = 0, n_stamps: int = 0):
    wl, pair = pair_for(name, seed, width, height, n_stamps)
    cfg = O.Config.from_workload(wl)
    return O.match_pair(cfg, pair, c_out=wl.cov_half)


def norm_err_M(Mg, Mo):
    """max |dM_ij| / sqrt(M_ii M_jj) over stamps (scale-free Gram error)."""
    d = np.sqrt(np.abs(np.einsum("sii->si", Mo)))
    den = d[:, :, None] * d[:, None, :]
    den[den == 0] = 1.0
    return float(np.max(np.abs(Mg - Mo) / den))
