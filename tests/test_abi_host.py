"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/adjwave.h declares, validates arguments before any
device work, and its host utilities agree with the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import blur as obl
from oracle import filters as ofl
from oracle import wavelet as owv
from paper_1707_02018_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "adjwave.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^(?:aw_status|const char\*)\s+(\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    names = header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) - {"aw_last_error", "aw_batch_last_error"} == set(_lib.SIGNATURES)


def _wave(rows=64, cols=48, levels=3, L=8, bc=1, lo=None):
    w = _lib.Wavelet()
    w.rows, w.cols, w.levels, w.filter_len, w.bc = rows, cols, levels, L, bc
    for k, v in enumerate(ofl.by_taps(L) if lo is None else lo):
        w.lo[k] = v
    return w


@pytest.mark.parametrize("taps", [2, 4, 8, 16])
def test_daubechies_matches_oracle(lib, taps):
    out = (ctypes.c_double * taps)()
    assert lib.aw_daubechies(taps, out) == _lib.OK
    np.testing.assert_allclose(np.array(out[:]), ofl.by_taps(taps), atol=1e-13)


def test_gaussian_psf_matches_oracle(lib):
    for sigma, r in [(2.0, 4), (3.0, 7), (1.3, 4), (4.0, 12), (0.5, 0)]:
        out = (ctypes.c_double * (2 * r + 1))()
        assert lib.aw_gaussian_psf(sigma, r, out) == _lib.OK
        np.testing.assert_allclose(np.array(out[:]), obl.gaussian_taps(sigma, r), atol=1e-15)


@pytest.mark.parametrize("bc,mode", [(0, "zpd"), (1, "sym"), (2, "per"), (3, "per_ext")])
@pytest.mark.parametrize("L", [2, 8, 16])
def test_layout_matches_oracle(lib, bc, mode, L):
    for rows, cols, J in [(256, 256, 3), (2048, 2048, 4), (96, 160, 5), (32, 32, 4), (5, 9, 2)]:
        if mode == "per" and (rows % 2 ** J or cols % 2 ** J):
            continue
        w = _wave(rows, cols, J, L, bc)
        n = ctypes.c_int64()
        sr = (ctypes.c_int32 * (J + 1))()
        sc = (ctypes.c_int32 * (J + 1))()
        assert lib.aw_wavelet_layout(ctypes.byref(w), ctypes.byref(n), sr, sc) == _lib.OK
        ref_n, ref_r, ref_c = owv.layout(rows, cols, L, mode, J)
        assert n.value == ref_n
        assert list(sr) == ref_r and list(sc) == ref_c


def _einval(lib, w):
    n = ctypes.c_int64()
    st = lib.aw_wavelet_layout(ctypes.byref(w), ctypes.byref(n), None, None)
    return st == _lib.EINVAL and len(lib.aw_last_error()) > 0


def test_invalid_wavelet_descriptors(lib):
    assert _einval(lib, _wave(levels=0))
    assert _einval(lib, _wave(levels=9))
    assert _einval(lib, _wave(L=6))
    assert _einval(lib, _wave(bc=7))
    assert _einval(lib, _wave(rows=0))
    assert _einval(lib, _wave(rows=24, cols=24, levels=4, bc=2))  # odd size at a level
    bad = ofl.by_taps(8).copy()
    bad[0] += 1e-6
    assert _einval(lib, _wave(lo=bad))                          # not orthonormal
    assert lib.aw_wavelet_layout(None, None, None, None) == _lib.EINVAL
    w = _wave()
    assert lib.aw_wavelet_layout(ctypes.byref(w), None, None, None) == _lib.OK
    assert lib.aw_last_error() == b""


def test_entry_points_validate_before_launch(lib):
    """Invalid calls return EINVAL without touching the device (this test
    runs without a GPU)."""
    w = _wave()
    b = _lib.Blur()
    b.rows, b.cols, b.radius = 64, 48, 4
    for i, v in enumerate(obl.gaussian_taps(2.0, 4)):
        b.taps[i] = v
    dummy = ctypes.c_void_p(0x1000)
    ws = ctypes.c_void_p(0x2000)
    W, B = ctypes.byref(w), ctypes.byref(b)
    assert lib.wavelet_synth(W, 0, 1, None, dummy, ws, 1 << 30, None) == _lib.EINVAL
    assert lib.wavelet_synth(W, 5, 1, dummy, dummy, ws, 1 << 30, None) == _lib.EINVAL
    assert lib.wavelet_synth(W, 0, 0, dummy, dummy, ws, 1 << 30, None) == _lib.EINVAL
    assert lib.wavelet_synth(W, 0, 1, dummy, dummy, ws, 16, None) == _lib.EINVAL  # small ws
    assert lib.wavelet_synth_adjoint(W, 0, 1, dummy, dummy, None, 0, None) == _lib.EINVAL
    b.radius = 13
    assert lib.blur(B, 0, 1, dummy, ws, None) == _lib.EINVAL
    b.radius = 4
    assert lib.blur(B, 0, 1, dummy, dummy, None) == _lib.EINVAL  # aliasing
    b2 = _lib.Blur()
    b2.rows, b2.cols, b2.radius = 32, 48, 0
    b2.taps[0] = 1.0
    assert lib.aw_apply_A(W, ctypes.byref(b2), 0, 1, dummy, dummy, ws, 1 << 30,
                          None) == _lib.EINVAL  # size mismatch
    st = _lib.FistaState()
    st.x = st.y = st.resid = 0x3000
    st.k, st.t = 0, 1.0
    assert lib.fista_step(W, B, 0, 1, dummy, 1.0, 2e-5, ctypes.byref(st), 0, ws, 1 << 30,
                          None) == _lib.EINVAL  # k = 0
    st.k = 1
    assert lib.fista_step(W, B, 0, 1, dummy, 0.0, 2e-5, ctypes.byref(st), 0, ws, 1 << 30,
                          None) == _lib.EINVAL  # L = 0
    assert lib.fista_step_noalloc(W, B, 0, 1, dummy, 0.0, 2e-5, ctypes.byref(st), 0,
                                  None) == _lib.EINVAL  # L = 0
    assert lib.fista_step_noalloc(W, B, 0, 1, dummy, 1.0, 2e-5, None, 0,
                                  None) == _lib.EINVAL  # no state
    # a problem whose workspace exceeds the 64 MiB static scratch
    wb, bb = _lib.Wavelet(), _lib.Blur()
    ctypes.memmove(ctypes.byref(wb), ctypes.byref(w), ctypes.sizeof(w))
    wb.rows = wb.cols = 4096
    bb.rows = bb.cols = 4096
    bb.radius = 4
    for i, v in enumerate(obl.gaussian_taps(2.0, 4)):
        bb.taps[i] = v
    assert lib.fista_step_noalloc(ctypes.byref(wb), ctypes.byref(bb), 0, 1, dummy, 1.0, 2e-5,
                                  ctypes.byref(st), 0, None) == _lib.EINVAL
    assert b"static scratch" in lib.aw_last_error()
    S = ctypes.byref(st)
    assert lib.aw_fista_update(W, 0, 1, dummy, 1.0, 2e-5, None, 0, ws, 1 << 30,
                               None) == _lib.EINVAL  # no state
    assert lib.aw_fista_update(W, 0, 1, None, 1.0, 2e-5, S, 0, ws, 1 << 30,
                               None) == _lib.EINVAL  # no gradient
    assert lib.aw_fista_update(W, 0, 1, dummy, 1.0, -1.0, S, 0, ws, 1 << 30,
                               None) == _lib.EINVAL  # lambda < 0
    assert lib.aw_fista_update(W, 0, 1, dummy, 1.0, 2e-5, S, 0, ws, 16,
                               None) == _lib.EINVAL  # small workspace
    st.gradient = 5
    assert lib.aw_fista_update(W, 0, 1, dummy, 1.0, 2e-5, S, 0, ws, 1 << 30,
                               None) == _lib.EINVAL  # unknown gradient map
    st.gradient = 0
    assert st.k == 1 and st.t == 1.0  # a rejected call advances nothing
    assert lib.conv_adjoint_pair(0, 1, 0, 5, dummy, dummy, None, ws, None, None,
                                 None) == _lib.EINVAL
    assert lib.conv_adjoint_pair(0, 1, 3, 5, dummy, ws, None, ws, None, None,
                                 None) == _lib.EINVAL  # aliasing


def test_workspace_size_grows_with_batch(lib):
    w = _wave(2048, 2048, 4, 8, 1)
    b = _lib.Blur()
    b.rows, b.cols, b.radius = 2048, 2048, 7
    n1, n4 = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.aw_workspace_size(ctypes.byref(w), ctypes.byref(b), 0, 1, ctypes.byref(n1)) == 0
    assert lib.aw_workspace_size(ctypes.byref(w), ctypes.byref(b), 0, 4, ctypes.byref(n4)) == 0
    # at least a_1..a_3, one image and one coefficient vector
    _, sr, sc = owv.layout(2048, 2048, 8, "sym", 4)
    floor = 4 * (sum(sr[j] * sc[j] for j in range(1, 4)) + 2048 * 2048 + 4352319)
    assert n1.value >= floor
    assert n4.value >= 4 * floor


def test_batch_plan_validates_before_device_work(lib):
    plan = ctypes.c_void_p()
    w = (_lib.Wavelet * 2)(_wave(), _wave(bc=3))
    b = (_lib.Blur * 2)()
    for i in range(2):
        b[i].rows, b[i].cols, b[i].radius = 64, 48, 0
        b[i].taps[0] = 1.0
    assert lib.aw_batch_create(0, w, b, ctypes.byref(plan)) == _lib.EINVAL
    assert lib.aw_batch_create(2, w, b, ctypes.byref(plan)) == _lib.EUNSUPPORTED
    assert b"periodic extension" in lib.aw_batch_last_error()
    w2 = (_lib.Wavelet * 1)(_wave(rows=5, cols=9, levels=1))  # sym level shorter than L - 1
    b2 = (_lib.Blur * 1)()
    b2[0].rows, b2[0].cols, b2[0].radius = 5, 9, 0
    b2[0].taps[0] = 1.0
    assert lib.aw_batch_create(1, w2, b2, ctypes.byref(plan)) == _lib.EUNSUPPORTED


def test_cnn_entry_points_validate(lib):
    pk, act, ws = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.aw_cnn_sizes(4, 512, 512, ctypes.byref(pk), ctypes.byref(act),
                            ctypes.byref(ws)) == _lib.OK
    assert act.value == 4 * 512 * 512 * 5 * 32 * 2
    # packed: BF16 forward + mirrored copies of four mid layers, output layer padded to 32
    assert pk.value == 9 * 32 * 2 + 128 + 4 * (2 * 9216 * 2 + 128) + 9216 * 2 + 128 + 9 * 32 * 2
    assert ws.value >= 9248 * 4
    assert lib.aw_cnn_sizes(0, 8, 8, None, None, None) == _lib.EINVAL
    assert lib.aw_cnn_sizes(64, 4096, 4096, None, None, None) == _lib.EINVAL  # index range
    d = ctypes.c_void_p(0x1000)
    assert lib.aw_cnn_pack(None, d, None) == _lib.EINVAL
    assert lib.aw_cnn_forward(d, 1, 8, 8, d, d, d, None) == _lib.EINVAL       # u aliases b
    assert lib.aw_cnn_forward(d, 1, 0, 8, d, d, ctypes.c_void_p(0x2000), None) == _lib.EINVAL
    e = ctypes.c_void_p(0x2000)
    assert lib.aw_cnn_backward(d, 1, 8, 8, d, d, d, e, d, d, 16, None) == _lib.EINVAL  # ws
    assert lib.aw_cnn_backward(d, 1, 8, 8, d, d, d, d, d, d, 1 << 30, None) == _lib.EINVAL
    assert lib.aw_adam_step(d, d, d, d, 10, 0, 1e-3, 0.9, 0.999, 1e-8, None) == _lib.EINVAL
    assert lib.aw_adam_step(d, d, d, d, 10, 1, 1e-3, 1.0, 0.999, 1e-8, None) == _lib.EINVAL
    assert lib.aw_adam_step(d, d, d, d, 10, 1, -1.0, 0.9, 0.999, 1e-8, None) == _lib.EINVAL
    assert lib.aw_soft_threshold(10, d, -1.0, d, None) == _lib.EINVAL
    assert lib.aw_sq_error(10, d, d, 1.0, None, d, d, 0, None) == _lib.EINVAL  # ws too small
    n = ctypes.c_size_t()
    assert lib.aw_sq_error_workspace(100000, ctypes.byref(n)) == _lib.OK and n.value >= 8


def test_cdf97_matches_oracle(lib):
    """The native CDF 9/7 construction against the oracle's (independent code
    of the same factorisation)."""
    hs, ha = (ctypes.c_double * 10)(), (ctypes.c_double * 10)()
    assert lib.aw_cdf97(hs, ha) == _lib.OK
    ref_s, ref_a = ofl.cdf97()
    np.testing.assert_allclose(np.array(hs[:]), ref_s, atol=1e-15)
    np.testing.assert_allclose(np.array(ha[:]), ref_a, atol=1e-15)
    assert lib.aw_cdf97(None, ha) == _lib.EINVAL


def _bior(rows=64, cols=64, levels=3, bc=1, hs=None, ha=None, flag=1):
    ref_s, ref_a = ofl.cdf97()
    w = _lib.Wavelet()
    w.rows, w.cols, w.levels, w.filter_len, w.bc = rows, cols, levels, 10, bc
    for k in range(10):
        w.lo[k] = float((ref_s if hs is None else hs)[k])
        w.lo_analysis[k] = float((ref_a if ha is None else ha)[k])
    w.biorthogonal = flag
    return w


@pytest.mark.parametrize("bc,mode", [(0, "zpd"), (1, "sym"), (2, "per"), (3, "per_ext")])
def test_biorthogonal_layout_and_validation(lib, bc, mode):
    for rows, cols, J in [(256, 256, 3), (96, 160, 4), (18, 10, 1)]:
        if mode == "per" and (rows % 2 ** J or cols % 2 ** J):
            continue
        w = _bior(rows, cols, J, bc)
        n = ctypes.c_int64()
        sr = (ctypes.c_int32 * (J + 1))()
        sc = (ctypes.c_int32 * (J + 1))()
        assert lib.aw_wavelet_layout(ctypes.byref(w), ctypes.byref(n), sr, sc) == _lib.OK
        ref_n, ref_r, ref_c = owv.layout(rows, cols, 10, mode, J)
        assert n.value == ref_n and list(sr) == ref_r and list(sc) == ref_c
    ref_s, ref_a = ofl.cdf97()
    assert _einval(lib, _bior(flag=0))                    # the pair is not orthonormal
    assert _einval(lib, _bior(flag=2))
    assert _einval(lib, _bior(ha=np.roll(ref_a, 1)))      # shifted: not biorthogonal
    bad = ref_s.copy()
    bad[4] += 1e-6
    assert _einval(lib, _bior(hs=bad))


def test_blur_dct_plan_validates_before_device_work(lib):
    """Invalid DCT-blur plans are refused on the host (no device memory)."""
    g = obl.gaussian_taps(2.0, 4)
    arr = (ctypes.c_double * len(g))(*g)
    plan = ctypes.c_void_p()
    assert lib.aw_blur_dct_create(48, 64, 4, arr, 0, ctypes.byref(plan)) == _lib.EUNSUPPORTED
    assert lib.aw_blur_dct_create(64, 8192, 4, arr, 0, ctypes.byref(plan)) == _lib.EUNSUPPORTED
    asym = g.copy()
    asym[0] += 1e-3
    arr2 = (ctypes.c_double * len(asym))(*asym)
    assert lib.aw_blur_dct_create(64, 64, 4, arr2, 0, ctypes.byref(plan)) == _lib.EUNSUPPORTED
    assert lib.aw_blur_dct_create(64, 64, -1, arr, 0, ctypes.byref(plan)) == _lib.EINVAL
    assert lib.aw_blur_dct_create(64, 64, 4, None, 0, ctypes.byref(plan)) == _lib.EINVAL
    assert lib.aw_blur_dct_create(64, 64, 4, arr, 7, ctypes.byref(plan)) == _lib.EINVAL
    assert lib.aw_blur_dct_create(64, 64, 4, arr, 0, None) == _lib.EINVAL
    assert plan.value is None
    assert lib.aw_blur_dct_destroy(None) == _lib.OK
