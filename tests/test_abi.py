"""Host-only checks of the C ABI: the library loads without a GPU, exports every
symbol include/cr.h declares, and rejects bad arguments before any HIP call."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    import paper_1407_7220_amd as cr
    return cr, cr._lib


def _declared():
    text = open(os.path.join(ROOT, "include", "cr.h")).read()
    return sorted(set(re.findall(r"\b(cr_[a-z_]+)\s*\(", text)))


def test_header_symbols_exported():
    cr, lib = _lib()
    names = _declared()
    assert "cr_solve" in names and "cr_pairwise_step" in names and "cr_init" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(cr.EXPORTED) == set(names)


def test_status_strings_and_defaults():
    cr, lib = _lib()
    assert lib.cr_status_string(0) == b"CR_OK"
    assert lib.cr_status_string(5) == b"CR_NOT_CONVERGED"
    p = cr._CParams()
    assert lib.cr_params_default(ctypes.byref(p)) == 0
    assert p.gamma == 1e-3 and p.c == 4.0 and p.step_scale == 0.5 and p.precision == 0
    assert lib.cr_params_default(None) == cr.ERR_ARG


def test_workspace_bytes_validation_and_growth():
    cr, lib = _lib()
    b1 = cr.workspace_bytes(2000, 10)
    b2 = cr.workspace_bytes(4000, 10)
    # dominated by the N x N multiplier array theta (FP64 by default)
    assert b1 >= 2000 * 2000 * 8 and b2 >= 4000 * 4000 * 8
    assert 3.3 < b2 / b1 < 4.5
    assert cr.workspace_bytes(1000, 10, cr.Params(precision=cr.F32)) < b1
    for N, n, status in [(1, 2, cr.ERR_ARG), (10, 0, cr.ERR_ARG), (10, 32, cr.ERR_UNSUPPORTED)]:
        with pytest.raises(cr.CRError) as e:
            cr.workspace_bytes(N, n)
        assert e.value.status == status
    with pytest.raises(cr.CRError):
        cr.workspace_bytes(10, 2, cr.Params(gamma=0.0))
    with pytest.raises(cr.CRError):
        cr.workspace_bytes(10, 2, cr.Params(c=1.0))
    with pytest.raises(cr.CRError):
        cr.workspace_bytes(10, 2, cr.Params(step_scale=1.5))
    with pytest.raises(cr.CRError):
        cr.workspace_bytes(10, 2, cr.Params(precision=7))
    with pytest.raises(cr.CRError):
        cr.workspace_bytes(10, 2, cr.Params(deterministic=2))
    assert cr.workspace_bytes(10, 2, cr.Params(deterministic=1)) == cr.workspace_bytes(10, 2)


def test_init_rejects_before_touching_the_gpu():
    cr, lib = _lib()
    p = cr.Params().to_c()
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)
    need = cr.workspace_bytes(50, 3)
    # null output handle, null inputs, bad sizes, small workspace
    assert lib.cr_init(None, 50, 3, ctypes.byref(p), fake, fake, fake, need, None) == cr.ERR_ARG
    assert lib.cr_init(ctypes.byref(h), 50, 3, ctypes.byref(p), None, fake, fake, need, None) == cr.ERR_ARG
    assert lib.cr_init(ctypes.byref(h), 1, 3, ctypes.byref(p), fake, fake, fake, need, None) == cr.ERR_ARG
    assert lib.cr_init(ctypes.byref(h), 50, 40, ctypes.byref(p), fake, fake, fake, need, None) == cr.ERR_UNSUPPORTED
    assert lib.cr_init(ctypes.byref(h), 50, 3, ctypes.byref(p), fake, fake, fake, need - 1, None) == cr.ERR_NOMEM
    assert b"workspace" in lib.cr_last_error(None)
    assert h.value is None
    bad = cr.Params(tau1=-1.0).to_c()
    assert lib.cr_init(ctypes.byref(h), 50, 3, ctypes.byref(bad), fake, fake, fake, need, None) == cr.ERR_ARG
    # entry points that take a context reject NULL
    assert lib.cr_pairwise_step(None, 0, fake, fake, fake, fake, 1.0, 2.0) == cr.ERR_ARG
    assert lib.cr_run(None, fake, fake, None) == cr.ERR_ARG
    cnt = ctypes.c_int32(0)
    assert lib.cr_get_outer_history(None, 0, None, None, ctypes.byref(cnt)) == cr.ERR_ARG
    assert lib.cr_destroy(None) == cr.OK
    assert lib.cr_solve(fake, fake, 50, 3, ctypes.byref(p), None, fake, fake, need, None, None) == cr.ERR_ARG


def test_product_package_has_no_oracle_dependency():
    pkg = os.path.join(ROOT, "paper_1407_7220_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "cr_oracle" not in text and "libcr_oracle" not in text, f


def test_batch_arguments_rejected_on_host():
    cr, lib = _lib()
    p = cr.Params().to_c()
    arr = (cr._CProblem * 2)()
    arr[0] = cr._CProblem(100, 3, 0, 0x1000, 0x1000, 0x1000, 0x1000)
    arr[1] = cr._CProblem(50, 40, 0, 0x1000, 0x1000, 0x1000, 0x1000)
    out = ctypes.c_size_t(0)
    assert lib.cr_batch_workspace_bytes(arr, 0, ctypes.byref(p), ctypes.byref(out)) == cr.ERR_ARG
    assert lib.cr_batch_workspace_bytes(arr, 2, ctypes.byref(p), ctypes.byref(out)) == cr.ERR_UNSUPPORTED
    assert lib.cr_batch_workspace_bytes(arr, 1, ctypes.byref(p), ctypes.byref(out)) == cr.OK
    one = out.value
    assert one >= cr.workspace_bytes(100, 3)
    mixed = cr.Params(precision=cr.MIXED_BF16).to_c()
    assert lib.cr_batch_workspace_bytes(arr, 1, ctypes.byref(mixed), ctypes.byref(out)) == cr.ERR_UNSUPPORTED
    h = ctypes.c_void_p()
    assert lib.cr_batch_init(ctypes.byref(h), arr, 1, ctypes.byref(p), ctypes.c_void_p(0x1000), one - 1, None) == cr.ERR_NOMEM
    arr[0].y_dev = None
    assert lib.cr_batch_init(ctypes.byref(h), arr, 1, ctypes.byref(p), ctypes.c_void_p(0x1000), one, None) == cr.ERR_ARG
    assert lib.cr_batch_run(None, None, None) == cr.ERR_ARG
    running = ctypes.c_int32(0)
    assert lib.cr_batch_start(None) == cr.ERR_ARG
    assert lib.cr_batch_advance(None, 1, ctypes.byref(running)) == cr.ERR_ARG
    assert lib.cr_batch_finish(None, None, None) == cr.ERR_ARG
    assert lib.cr_batch_destroy(None) == cr.OK


def test_autotune_cache_roundtrip(tmp_path, monkeypatch):
    """Tuner cache: keys on (n, precision, power-of-two N bucket), JSON round trip,
    lookup misses give None and tile_rows_for falls back to 0 when tuning is off."""
    import paper_1407_7220_amd as cr
    from paper_1407_7220_amd import autotune as at
    import numpy as np
    monkeypatch.setenv("CR_TILE_CACHE", str(tmp_path / "cache.json"))
    assert at.bucket(5000) == 4871 and at.bucket(4334) == 4096 and at.bucket(2) == 2
    assert at.bucket(4096) == 4096 and at.bucket(6000) == 5793
    assert at.key(5000, 10, cr.F32) == "n10-f32-N4871"
    assert at.key(20000, 4, cr.MIXED_BF16) == "n4-mixed_bf16-N19484"
    assert at.lookup(5000, 10, cr.F32) is None
    at.save_cache({at.key(5000, 10, cr.F32): {"tile_rows": 512}})
    assert at.lookup(4900, 10, cr.F32) == 512
    assert at.lookup(4300, 10, cr.F32) is None
    assert at.lookup(5000, 10, cr.F64) is None
    X = np.zeros((5000, 10))
    assert at.tile_rows_for(X, None, cr.F32, tune_if_missing=False) == 512
    assert at.tile_rows_for(X, None, cr.F64, tune_if_missing=False) == 0


def test_diff_workspace_and_argument_checks():
    """cr_diff_workspace_bytes: host-side checks of the differentiable form and
    the theta store's growth with the number of ALCC iterations."""
    import paper_1407_7220_amd as cr
    p = cr.Params(precision=cr.F32, inner_iters=20, max_outer=10)
    b10 = cr.diff_workspace_bytes(2000, 10, p, 20)
    b2 = cr.diff_workspace_bytes(2000, 10, cr.Params(precision=cr.F32, inner_iters=20, max_outer=2), 20)
    theta_bytes = 2048 * 2048 * 4
    assert b10 - b2 >= 8 * theta_bytes
    assert b10 - b2 < 8 * theta_bytes + 64 * 2048 * 11 * 8 + (1 << 20)
    # finer checkpoints cost only O(N n) per checkpoint
    b1 = cr.diff_workspace_bytes(2000, 10, p, 1)
    assert b10 < b1 < b10 + 10 * 20 * 2 * 2048 * 11 * 8 + (1 << 20)
    with pytest.raises(cr.CRError) as e:
        cr.diff_workspace_bytes(2000, 10, cr.Params(precision=cr.F32, inner_iters=0), 20)
    assert e.value.status == 1
    with pytest.raises(cr.CRError) as e:
        cr.diff_workspace_bytes(2000, 10, p, 0)
    assert e.value.status == 1
    with pytest.raises(cr.CRError) as e:
        cr.diff_workspace_bytes(2000, 10, cr.Params(precision=cr.MIXED_BF16, inner_iters=5), 20)
    assert e.value.status == 7


def test_eval_workspace_and_argument_checks():
    """cr_eval_workspace_bytes / cr_eval: host-side checks (no device pointer is
    touched when an argument is rejected)."""
    import ctypes
    import paper_1407_7220_amd as cr
    b = cr.eval_workspace_bytes(1000, 20)
    assert b >= 1024 * 24 * 8                      # 32-plane tiles of [xi d 0..] rows, 4 ceil((n+1)/4) slots
    assert b < 1024 * 24 * 8 + 4096
    for N, n, status in ((0, 3, 1), (10, 0, 1), (10, 32, 7)):
        with pytest.raises(cr.CRError) as e:
            cr.eval_workspace_bytes(N, n)
        assert e.value.status == status
    fake = ctypes.c_void_p(0x1000)
    lib = cr._lib
    # NULL operands, negative M, too small a workspace: rejected before any launch
    assert lib.cr_eval(None, fake, fake, 10, 3, fake, 5, fake, None, fake, 1 << 20, None) == 1
    assert lib.cr_eval(fake, fake, fake, 10, 3, fake, -1, fake, None, fake, 1 << 20, None) == 1
    assert lib.cr_eval(fake, fake, fake, 10, 3, fake, 5, fake, None, fake, 16, None) == 2
    assert b"workspace" in lib.cr_last_error(None)
    assert lib.cr_eval(fake, fake, fake, 10, 40, fake, 5, fake, None, fake, 1 << 20, None) == 7
    # M = 0 is a no-op (nothing launched)
    assert lib.cr_eval(fake, fake, fake, 10, 3, None, 0, None, None, fake, 1 << 20, None) == 0


def test_papg_workspace_and_argument_checks():
    """cr_papg_workspace_bytes / cr_papg: host-side checks before any launch."""
    import ctypes
    import paper_1407_7220_amd as cr
    p = cr.Params(precision=cr.F64, inner_iters=20, max_outer=3)
    b = cr.papg_workspace_bytes(100, 5, p, cr.PapgParams(K=2, iters=3))
    assert b >= 2 * 100 * 100 * 8                  # two N x N multiplier arrays
    for N, n, K, it, status in ((100, 5, 3, 3, 1), (100, 5, 0, 3, 1), (100, 5, 100, 3, 1), (100, 5, 2, 0, 1),
                                (100, 40, 2, 3, 7)):
        with pytest.raises(cr.CRError) as e:
            cr.papg_workspace_bytes(N, n, p, cr.PapgParams(K=K, iters=it))
        assert e.value.status == status
    with pytest.raises(cr.CRError) as e:
        cr.papg_workspace_bytes(100, 5, cr.Params(precision=cr.MIXED_BF16), cr.PapgParams(K=2))
    assert e.value.status == 7
    with pytest.raises(cr.CRError) as e:
        cr.papg_workspace_bytes(100, 5, p, cr.PapgParams(K=2, method=2))
    assert e.value.status == 1
    with pytest.raises(cr.CRError) as e:
        cr.papg_workspace_bytes(100, 5, p, cr.PapgParams(K=2, power_iters=-1))
    assert e.value.status == 1
    fake = ctypes.c_void_p(0x1000)
    cp, cpp = p.to_c(), cr.PapgParams(K=2, iters=3).to_c()
    lib = cr._lib
    assert lib.cr_papg(None, fake, 100, 5, ctypes.byref(cp), ctypes.byref(cpp), fake, fake, None, None, None, fake,
                       1 << 30, None, None) == 1
    assert lib.cr_papg(fake, fake, 100, 5, ctypes.byref(cp), ctypes.byref(cpp), fake, fake, None, None, None, fake,
                       16, None, None) == 2
    assert b"workspace" in lib.cr_last_error(None)


def test_eval_noalloc_rejects_on_host():
    """Argument and size checks of the allocation-free estimator entry point
    run before any HIP call: 174752 planes at n = 20 fit its 32 MiB scratch,
    174753 do not."""
    cr, lib = _lib()
    fake = ctypes.c_void_p(0x1000)
    assert lib.cr_eval_noalloc(None, fake, fake, 10, 3, fake, 5, fake, None, None) == cr.ERR_ARG
    assert lib.cr_eval_noalloc(fake, fake, fake, 0, 3, fake, 5, fake, None, None) == cr.ERR_ARG
    assert lib.cr_eval_noalloc(fake, fake, fake, 10, 32, fake, 5, fake, None, None) == cr.ERR_UNSUPPORTED
    assert lib.cr_eval_noalloc(fake, fake, fake, 174753, 20, fake, 5, fake, None, None) == cr.ERR_NOMEM
    assert b"static scratch" in lib.cr_last_error(None)
    assert lib.cr_eval_noalloc(fake, fake, fake, 1048577, 3, fake, 5, fake, None, None) == cr.ERR_NOMEM
    # within the limit and M = 0: nothing to do, no HIP call
    assert lib.cr_eval_noalloc(fake, fake, fake, 174752, 20, None, 0, None, None, None) == cr.OK
    assert lib.cr_eval_noalloc(fake, fake, fake, 1048576, 3, None, 0, None, None, None) == cr.OK
