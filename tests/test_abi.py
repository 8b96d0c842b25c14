"""The C-ABI library loads, exports every symbol the header declares, and
rejects invalid arguments on the host before any launch (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2204_08183_amd import survscan as ss

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "survscan.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ss_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(ss.LIB_PATH):
        from paper_2204_08183_amd import build
        build.build()
    return ss.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(ss.SIGNATURES), "binding and header disagree"


def test_status_strings(lib):
    for code in (ss.SS_OK, ss.SS_EINVAL, ss.SS_EWORKSPACE, ss.SS_EUNSUPPORTED,
                 ss.SS_EDEVICE, 12345):
        assert isinstance(ss.status_string(code), str)
    assert ss.status_string(ss.SS_OK) == "ok"


def test_sizes(lib):
    assert lib.ss_chunk_count(1) == 1
    assert lib.ss_chunk_count(ss.CHUNK) == 1
    assert lib.ss_chunk_count(ss.CHUNK + 1) == 2
    assert lib.ss_workspace_bytes(ss.COX, 1000) > 0
    assert lib.ss_workspace_bytes(ss.FINE_GRAY, 10**6) >= lib.ss_workspace_bytes(ss.COX, 1000)
    assert lib.ss_workspace_bytes(7, 1000) == 0
    assert lib.ss_prepare_workspace_bytes(1000, 10, 500) > 0
    assert lib.ss_prepare_workspace_bytes(0, 10, 500) == 0


def _fake(addr=0x100000):
    return ctypes.c_void_p(addr)


def test_invalid_arguments_rejected_before_launch(lib):
    f = _fake()
    big = 1 << 30
    # unknown model
    assert lib.ss_grad_hess(5, 10, 2, 0, f, f, f, f, f, f, f, None, f, f, f, f, big,
                            None) == ss.SS_EUNSUPPORTED
    # n < 1, j out of range, null e
    assert lib.ss_grad_hess(0, 0, 2, 0, f, f, f, None, None, f, f, None, f, f, f, f, big,
                            None) == ss.SS_EINVAL
    assert lib.ss_grad_hess(0, 10, 2, 2, f, f, f, None, None, f, f, None, f, f, f, f, big,
                            None) == ss.SS_EINVAL
    assert lib.ss_grad_hess(0, 10, 2, 0, None, f, f, None, None, f, f, None, f, f, f, f,
                            big, None) == ss.SS_EINVAL
    # Fine-Gray without its weights
    assert lib.ss_grad_hess(1, 10, 2, 0, f, f, f, None, None, f, f, None, f, f, f, f, big,
                            None) == ss.SS_EINVAL
    # workspace too small or misaligned
    assert lib.ss_grad_hess(0, 10, 2, 0, f, f, f, None, None, f, f, None, f, f, f, f, 16,
                            None) == ss.SS_EWORKSPACE
    assert lib.ss_grad_hess(0, 10, 2, 0, f, f, f, None, None, f, f, None, f, f, f,
                            _fake(0x100008), big, None) == ss.SS_EWORKSPACE
    # penalties
    assert lib.ss_ccd_update(9, 1.0, 10, 2, 0, f, f, f, f, f, f, f, f, None,
                             None) == ss.SS_EUNSUPPORTED
    assert lib.ss_ccd_update(1, 0.0, 10, 2, 0, f, f, f, f, f, f, f, f, None,
                             None) == ss.SS_EINVAL
    assert lib.ss_ccd_sweep(0, 0, 0.0, 10, 2, 1, 0, f, f, f, f, None, None, f, f, None, f,
                            f, f, f, f, None, f, big, None) == ss.SS_EINVAL
    # prepare: bad sizes, missing outputs, nnz > 2^31 - 1
    assert lib.ss_prepare(0, 0, 1, 0, f, f, f, f, None, f, f, f, f, f, f, None, f, None,
                          None, f, big, None) == ss.SS_EINVAL
    assert lib.ss_prepare(0, 10, 1, 1 << 31, f, f, f, f, None, f, f, f, f, f, f, None, f,
                          None, None, f, big, None) == ss.SS_EINVAL
    assert lib.ss_prepare(1, 10, 1, 5, f, f, f, f, None, f, f, f, f, f, f, None, f, None,
                          None, f, big, None) == ss.SS_EINVAL
    assert lib.ss_exp(0, f, f, None) == ss.SS_EINVAL
    assert lib.ss_gather(5, None, f, f, None) == ss.SS_EINVAL
    assert lib.ss_workspace_init(None, 100, None) == ss.SS_EWORKSPACE


def test_new_entry_points_validate_on_the_host(lib):
    f = _fake()
    big = 1 << 30
    # full gradient in eta: model, size, pointers, workspace
    assert lib.ss_eta_gradient_workspace_bytes(0) == 0
    ws = lib.ss_eta_gradient_workspace_bytes(1000)
    assert ws >= 4 * 8 * 1000  # four N-vectors of doubles at least
    assert lib.ss_eta_gradient(4, 1000, f, f, f, f, f, f, None, None, f, f, f, ws,
                               None) == ss.SS_EUNSUPPORTED
    assert lib.ss_eta_gradient(0, 0, f, f, f, f, f, f, None, None, f, f, f, ws,
                               None) == ss.SS_EINVAL
    assert lib.ss_eta_gradient(0, 1000, f, f, f, f, f, f, None, None, None, f, f, ws,
                               None) == ss.SS_EINVAL
    assert lib.ss_eta_gradient(1, 1000, f, f, f, f, f, f, None, None, f, f, f, ws,
                               None) == ss.SS_EINVAL
    assert lib.ss_eta_gradient(0, 1000, f, f, f, f, f, f, None, None, f, f, f, ws - 1,
                               None) == ss.SS_EWORKSPACE
    # X' (dl/deta): the workspace holds the eta-gradient workspace and the
    # per-span partials, at most 2 (n + p) of them
    for n, p in ((1000, 3), (1 << 27, 1), (1_000_000, 1000), (40_000, 30_000), (100, 10**6)):
        wb = lib.ss_beta_gradient_workspace_bytes(n, p)
        we = lib.ss_eta_gradient_workspace_bytes(n)
        assert we < wb <= we + 16 * (n + p) + 256, (n, p)
    assert lib.ss_beta_gradient_workspace_bytes(0, 5) == 0
    assert lib.ss_beta_gradient_workspace_bytes(5, 0) == 0
    wb = lib.ss_beta_gradient_workspace_bytes(1000, 3)
    # model n p inv_perm status eta e d8 d32 w g col rows vals chunk gb ge ll ws
    assert lib.ss_beta_gradient(4, 1000, 3, None, f, f, f, f, f, None, None, f, f, None, f, f,
                                None, f, f, wb, None) == ss.SS_EUNSUPPORTED
    assert lib.ss_beta_gradient(0, 1000, 0, None, f, f, f, f, f, None, None, f, f, None, f, f,
                                None, f, f, wb, None) == ss.SS_EINVAL
    assert lib.ss_beta_gradient(0, 1000, 3, None, f, f, f, f, f, None, None, f, f, None, None,
                                f, None, f, f, wb, None) == ss.SS_EINVAL
    assert lib.ss_beta_gradient(0, 1000, 3, None, f, f, f, f, f, None, None, f, f, None, f, f,
                                f, f, f, wb, None) == ss.SS_EINVAL   # grad_eta needs inv_perm
    assert lib.ss_beta_gradient(1, 1000, 3, None, f, f, f, f, f, None, None, f, f, None, f, f,
                                None, f, f, wb, None) == ss.SS_EINVAL
    assert lib.ss_beta_gradient(0, 1000, 3, None, f, f, f, f, f, None, None, f, f, None, f, f,
                                None, f, f, wb - 1, None) == ss.SS_EWORKSPACE
    # cross-validation: sizes, valued designs unsupported, Fine-Gray needs its
    # Kaplan-Meier arrays
    s = lib.ss_cv_stride(100_000)
    assert s >= 100_000 and s % 16384 == 0
    assert lib.ss_cv_stride(0) == 0
    assert lib.ss_cv_prepare_workspace_bytes(100_000, 100) == 100 * s // 8
    assert lib.ss_cv_prepare_workspace_bytes(100_000, 0) == 0
    assert lib.ss_cv_workspace_bytes(100) > 100 * 1024
    assert lib.ss_cv_workspace_bytes(0) == 0
    # perm status y d8 train col_ptr rows vals train_s d8_r d32_r xbits c_r w_r g_r g_h ws
    prep = [f, f, f, f, f, f, f, None, f, f, f, f, f, f, f, f, f, big, None]
    assert lib.ss_cv_prepare(5, 1000, 5, 10, *prep) == ss.SS_EUNSUPPORTED
    no_km = list(prep)
    no_km[14] = None
    assert lib.ss_cv_prepare(1, 1000, 5, 10, *no_km) == ss.SS_EINVAL
    no_y = list(prep)
    no_y[2] = None
    assert lib.ss_cv_prepare(1, 1000, 5, 10, *no_y) == ss.SS_EINVAL
    valued = list(prep)
    valued[7] = f
    assert lib.ss_cv_prepare(0, 1000, 5, 10, *valued) == ss.SS_EUNSUPPORTED
    assert lib.ss_cv_prepare(0, 1000, 5, 0, *prep) == ss.SS_EINVAL
    short = list(prep)
    short[-2] = 8
    assert lib.ss_cv_prepare(0, 1000, 5, 10, *short) == ss.SS_EWORKSPACE
    # eta e d8_r d32_r train_s xbits c_r w_r g_r beta delta g12 ws
    sw = [f] * 11 + [None, f, big, None]
    assert lib.ss_cv_sweep(5, 0, 0.0, 1000, 5, 10, 0, 5, *sw) == ss.SS_EUNSUPPORTED
    no_w = list(sw)
    no_w[7] = None
    assert lib.ss_cv_sweep(1, 0, 0.0, 1000, 5, 10, 0, 5, *no_w) == ss.SS_EINVAL
    assert lib.ss_cv_sweep(0, 0, 0.0, 1000, 5, 10, 0, 6, *sw) == ss.SS_EINVAL
    assert lib.ss_cv_sweep(0, 3, 0.0, 1000, 5, 10, 0, 5, *sw) == ss.SS_EUNSUPPORTED
    # a penalty needs a positive strength (l2: the prior variance; l1: gamma)
    assert lib.ss_cv_sweep(0, 2, 0.0, 1000, 5, 10, 0, 5, *sw) == ss.SS_EINVAL
    assert lib.ss_cv_sweep(0, 1, -1.0, 1000, 5, 10, 0, 5, *sw) == ss.SS_EINVAL
    assert lib.ss_cv_sweep(0, 0, 0.0, 1000, 5, 70000, 0, 5, *sw) == ss.SS_EINVAL
    small = sw[:-2] + [16, None]
    assert lib.ss_cv_sweep(0, 0, 0.0, 1000, 5, 10, 0, 5, *small) == ss.SS_EWORKSPACE
    assert lib.ss_cv_exp(1000, 0, f, f, f, None) == ss.SS_EINVAL
    # perm status eta e train_s d8 d32 d8_r d32_r w_r g_r g_h out
    ll = [f] * 13 + [None]
    assert lib.ss_cv_loglik(5, 1000, 10, *ll) == ss.SS_EUNSUPPORTED
    no_gh = list(ll)
    no_gh[11] = None
    assert lib.ss_cv_loglik(1, 1000, 10, *no_gh) == ss.SS_EINVAL
    # FP32 path: unknown accumulation
    assert lib.ss_grad_hess_mixed(0, 9, 10, 2, 0, f, f, f, None, None, f, f, None, f, f, f,
                                  f, big, None) == ss.SS_EINVAL


def test_binding_fails_loudly_without_the_library(monkeypatch, tmp_path):
    """No CPU fallback: with the library absent every call raises."""
    monkeypatch.setattr(ss, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(ss, "_lib", None)
    with pytest.raises(ss.SurvScanError):
        ss.load()
    with pytest.raises(ss.SurvScanError):
        ss.Problem("cox", [1.0, 2.0], [1, 0], [0, 1], [0], None, "cpu")


def test_tune_table_host_logic(lib):
    """The launch-shape table (no launch, no GPU): built-in rule, pinning,
    size buckets of ceil(log2 n), impossible choices, clearing."""
    G, S = ss.TUNE_GRAD_HESS, ss.TUNE_SWEEP
    ss.tune_clear()
    try:
        # the built-in rule: tiles of 2048 positions up to 1.5 M, 4096 above
        assert ss.tune_get(G, "cox", "f64", False, 1_000_000) == 8
        assert ss.tune_get(G, "cox", "f64", False, 3 << 19) == 8
        assert ss.tune_get(G, "cox", "f64", False, (3 << 19) + 1) == 16
        assert ss.tune_get(S, "fg", "f64", True, 1000) == 0
        assert not ss.tune_has(G, "cox", "f64", False, 1000)
        ss.tune_set(G, "cox", "f64", False, 1000, 32)
        # 513 ... 1024 share the bucket ceil(log2 n) = 10
        for n in (513, 1000, 1024):
            assert ss.tune_get(G, "cox", "f64", False, n) == 32
            assert ss.tune_has(G, "cox", "f64", False, n)
        assert ss.tune_get(G, "cox", "f64", False, 1025) == 8
        assert ss.tune_get(G, "cox", "f64", False, 512) == 8
        # other models, storages and designs are separate keys
        assert ss.tune_get(G, "fg", "f64", False, 1000) == 8
        assert ss.tune_get(G, "cox", "f32", False, 1000) == 8
        assert ss.tune_get(G, "cox", "f64", True, 1000) == 8
        ss.tune_set(S, "cox", "f64", False, 1000, 51208)
        assert ss.tune_get(S, "cox", "f64", False, 1000) == 51208
        for kind, model, storage, choice in ((G, "cox", "f64", 12), (S, "cox", "f64", 25612),
                                             (S, "fg", "f64", 51216), (S, "cox", "f32", 25616)):
            assert lib.ss_tune_set(kind, ss.MODELS[model], ss.STORAGES[storage], 0, 1000,
                                   choice) == ss.SS_EINVAL
        assert lib.ss_tune_set(7, 0, 0, 0, 1000, 8) == ss.SS_EINVAL
        assert lib.ss_tune_get(0, 5, 0, 0, 1000) == ss.SS_EINVAL
        assert lib.ss_tune_get(0, 0, 3, 0, 1000) == ss.SS_EINVAL
        assert lib.ss_tune_get(0, 0, 0, 0, 0) == ss.SS_EINVAL
        ss.tune_set(G, "cox", "f64", False, 1000, 0)   # removes the entry
        assert not ss.tune_has(G, "cox", "f64", False, 1000)
        ss.tune_clear()
        assert not ss.tune_has(S, "cox", "f64", False, 1000)
    finally:
        ss.tune_clear()


def test_autotune_rejects_bad_arguments(lib):
    choice = ctypes.c_int32(0)
    args = [None] * 11 + [None, 0]
    assert lib.ss_autotune_grad_hess(0, 0, 100, 1, 0, *args, 0, ctypes.byref(choice), None,
                                     None) == ss.SS_EINVAL
    assert lib.ss_autotune_grad_hess(0, 5, 100, 1, 0, *args, 10, ctypes.byref(choice), None,
                                     None) == ss.SS_EINVAL
    sargs = [None] * 18 + [None, 0]
    assert lib.ss_autotune_sweep(0, 1, 1.0, 100, 4, 2, 2, *sargs, 3, ctypes.byref(choice),
                                 None, None) == ss.SS_EINVAL
    assert lib.ss_autotune_sweep(0, 1, 0.0, 100, 4, 0, 2, *sargs, 3, ctypes.byref(choice),
                                 None, None) == ss.SS_EINVAL
