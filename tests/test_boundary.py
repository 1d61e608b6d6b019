"""The C interface without a GPU: the built library loads, exports every
function declared in include/psfm.h, and rejects bad arguments on the host
before anything is launched."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "psfm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(psfm_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1901_09999_amd import psfm
    if not os.path.exists(psfm.LIB_PATH):
        pytest.skip("libpsfm.so not built")
    return psfm.lib()


def test_header_declares_the_hot_path():
    names = declared_functions()
    for f in ("psfm_fit_stamps", "psfm_solve", "psfm_convolve_image", "psfm_propagate_variance",
              "psfm_subtract"):
        assert f in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_covers_header():
    from paper_1901_09999_amd import psfm
    assert set(psfm.exported_symbols()) == set(declared_functions())


def test_host_argument_checks(lib):
    from paper_1901_09999_amd import psfm
    cfg = psfm.CConfig()
    lib.psfm_config_default(C.byref(cfg))
    assert cfg.n_gauss == 3 and cfg.half_width == 10 and list(cfg.degree[:3]) == [6, 4, 2]
    assert abs(cfg.bad_frac - 0.2) < 1e-15 and cfg.max_iter == 3 and cfg.min_stamps == 3
    assert cfg.precision == 0 and cfg.refine == 1
    h = C.c_void_p()
    assert lib.psfm_create(None, C.byref(h)) == -1
    bad = psfm.CConfig()
    lib.psfm_config_default(C.byref(bad))
    bad.n_gauss = 0
    assert lib.psfm_create(C.byref(bad), C.byref(h)) == -1
    bad.n_gauss = 3
    bad.sigma[1] = -1.0
    assert lib.psfm_create(C.byref(bad), C.byref(h)) == -1
    lib.psfm_config_default(C.byref(bad))
    bad.half_width = 40
    assert lib.psfm_create(C.byref(bad), C.byref(h)) == -7
    lib.psfm_config_default(C.byref(bad))
    bad.degree[0] = 9                     # 55 + 15 + 6 terms: beyond the 64-column Gram
    assert lib.psfm_create(C.byref(bad), C.byref(h)) == -7
    lib.psfm_config_default(C.byref(bad))
    bad.precision = 3
    assert lib.psfm_create(C.byref(bad), C.byref(h)) == -7
    lib.psfm_config_default(C.byref(bad))
    bad.refine = 5
    assert lib.psfm_create(C.byref(bad), C.byref(h)) == -7
    for field, value, code in (("weight_mode", 2, -1), ("ortho_basis", 2, -1), ("flags", 2, -1),
                               ("fit_band_rows", 10, -7)):
        lib.psfm_config_default(C.byref(bad))
        setattr(bad, field, value)
        assert lib.psfm_create(C.byref(bad), C.byref(h)) == code, field
    assert lib.psfm_stamp_design_floats(None, 4) == 0
    assert lib.psfm_workspace_bytes(None, 10, 10, 1) == 0
    assert lib.psfm_fit_stamps(None, *([None] * 6), 10, 10, 10, None, 1, *([None] * 6), None, 0,
                               None) == -1
    assert lib.psfm_solve(None, 10, 10, None, 1, *([None] * 9), None, 0, None) == -1
    assert lib.psfm_convolve_image(None, None, None, None, 10, 10, 10, None, None, None, 0, None) == -1
    assert lib.psfm_fit_norm(None, None, None, 10, 10, 10, None, 1, None, None, None) == -1
    assert lib.psfm_solve_norm(None, 10, 10, None, 1, *([None] * 10), None, 0, None) == -1
    assert lib.psfm_quality_eval(None, None, None, None, None, 10, 10, 10, None, 1, None, 0.0, None,
                                 None, None) == -1
    assert lib.psfm_trace_mask(None, None, None, 10, 10, 10, 0.5, None, None) == -1


def test_stack_host_argument_checks(lib):
    """Homogenisation entry points reject bad arguments before any launch."""
    assert lib.psfm_envelope_psf(None, 1, 5, None, None, None) == -1
    assert lib.psfm_render_workspace_bytes(10, 0, 10, 1.0) == 0
    assert lib.psfm_render_workspace_bytes(10, 10, 10, -1.0) == 0
    assert lib.psfm_render_workspace_bytes(10, 64, 64, 2.0) > 0
    assert lib.psfm_render_target(None, 0, 1.0, 10, 10, 10, None, None, 0, None) == -1
    assert lib.psfm_stack_reject(0, None, None, None, 100, 10, 10, 10, 3.0, None, None) == -1
    assert lib.psfm_stack_combine(0, *([None] * 3), 100, 10, 10, 10, None, 0, *([None] * 6), 0,
                                  None) == -1
    for code in range(-8, 1):
        assert lib.psfm_status_string(code).decode()


def test_batch_host_argument_checks(lib):
    h = C.c_void_p()
    assert lib.psfm_batch_workspace_bytes(None, None, 1) == 0
    assert lib.psfm_batch_plan(None, None, 1, None, None, 0, None, None, C.byref(h)) == -1
    assert lib.psfm_batch_run(None, None) == -1
    assert lib.psfm_batch_run_stage(None, 0, None) == -1
    assert lib.psfm_batch_set_tuning(None, None) == -1
    assert lib.psfm_batch_graph_capture(None, None) == -1
    assert lib.psfm_batch_graph_launch(None, None) == -1
    assert lib.psfm_batch_destroy(None) == -1


def test_cnn_parameter_layout_matches_oracle(lib):
    from oracle import cnn_oracle as CO
    from paper_1901_09999_amd import cnn
    assert lib.psfm_cnn_param_count() == CO.n_params()
    assert cnn.layer_shapes() == CO.layer_shapes()
    assert lib.psfm_cnn_workspace_bytes(0) == 0 and lib.psfm_cnn_workspace_bytes(16) > 0
    assert lib.psfm_cnn_forward(None, None, 1, None, None, 0, None) == -1
    assert lib.psfm_cnn_loss_grad(None, None, None, None, 1, None, None, None, 0, None) == -1
    assert lib.psfm_cnn_loss_weights(None, None, None, None, 1, None, None) == -1
    assert lib.psfm_solve_stamps(None, 1, *([None] * 6), None) == -1
    assert lib.psfm_cholesky_workspace_bytes(0) == 0 and lib.psfm_cholesky_workspace_bytes(295) > 0
    assert lib.psfm_cholesky_solve(0, None, None, None, None, None, 0, None) == -1
    assert lib.psfm_cholesky_solve(600, *([None] * 4), None, 0, None) == -1


def test_batch_group_argument_checks(lib):
    """The batch-group entry points refuse bad arguments before any device call."""
    g = C.c_void_p()
    one = (C.c_void_p * 2)(C.c_void_p(16), C.c_void_p(16))      # the same plan twice
    stream = C.c_void_p(8)
    assert lib.psfm_batch_group_capture(None, 1, stream, C.byref(g)) == -1
    assert lib.psfm_batch_group_capture(one, 0, stream, C.byref(g)) == -1
    assert lib.psfm_batch_group_capture(one, 17, stream, C.byref(g)) == -1
    assert lib.psfm_batch_group_capture(one, 1, None, C.byref(g)) == -1
    assert lib.psfm_batch_group_capture(one, 1, stream, None) == -1
    assert lib.psfm_batch_group_capture(one, 2, stream, C.byref(g)) == -1
    nul = (C.c_void_p * 1)(None)
    assert lib.psfm_batch_group_capture(nul, 1, stream, C.byref(g)) == -1
    assert lib.psfm_batch_group_launch(None, stream) == -1
    assert lib.psfm_batch_group_destroy(None) == -1
