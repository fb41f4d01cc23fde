"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects bad arguments before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1811_11076_amd import _lib
from paper_1811_11076_amd.build import lib_path

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tsknn.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(tsk_[a-z_]+)\s*\(", text)))


needs_lib = pytest.mark.skipif(not os.path.exists(lib_path()),
                               reason="libtsknn.so not built (run the package build)")


@needs_lib
def test_exports_every_declared_symbol():
    lib = ctypes.CDLL(lib_path())
    names = _declared()
    assert "tsk_knn_query" in names and "tsk_index_build" in names
    for name in names:
        assert hasattr(lib, name), name
    # the binding's table covers the header
    assert set(_lib.SIGNATURES) == set(names)


@needs_lib
def test_version_and_error_text():
    lib = _lib.load()
    a, b = ctypes.c_int(), ctypes.c_int()
    assert lib.tsk_version(ctypes.byref(a), ctypes.byref(b)) == 0
    assert (a.value, b.value) == (0, 1)
    assert isinstance(lib.tsk_last_error(), bytes)


@needs_lib
def test_build_rejects_bad_arguments_before_device_work():
    lib = _lib.load()
    out = ctypes.c_void_p()
    off = np.array([0, 4, 8], np.int64)
    offp = off.ctypes.data_as(ctypes.c_void_p)
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    # null output
    assert lib.tsk_index_build(fake, offp, 2, 3, None, None, None) == _lib.TSK_ERR_INVALID_ARG
    # null values
    assert lib.tsk_index_build(None, offp, 2, 3, None, None, ctypes.byref(out)) == _lib.TSK_ERR_INVALID_ARG
    # unsupported dimension
    assert lib.tsk_index_build(fake, offp, 2, 0, None, None, ctypes.byref(out)) == _lib.TSK_ERR_UNSUPPORTED
    assert lib.tsk_index_build(fake, offp, 2, 33, None, None, ctypes.byref(out)) == _lib.TSK_ERR_UNSUPPORTED
    # zero-length series
    bad = np.array([0, 4, 4], np.int64)
    assert lib.tsk_index_build(fake, bad.ctypes.data_as(ctypes.c_void_p), 2, 3, None, None,
                               ctypes.byref(out)) == _lib.TSK_ERR_INVALID_ARG
    assert b"length 0" in lib.tsk_last_error()
    # too long
    long_ = np.array([0, 5000], np.int64)
    assert lib.tsk_index_build(fake, long_.ctypes.data_as(ctypes.c_void_p), 1, 3, None, None,
                               ctypes.byref(out)) == _lib.TSK_ERR_UNSUPPORTED
    # offsets[0] != 0 and empty database
    shifted = np.array([1, 4], np.int64)
    assert lib.tsk_index_build(fake, shifted.ctypes.data_as(ctypes.c_void_p), 1, 3, None, None,
                               ctypes.byref(out)) == _lib.TSK_ERR_INVALID_ARG
    assert lib.tsk_index_build(fake, offp, 0, 3, None, None, ctypes.byref(out)) == _lib.TSK_ERR_INVALID_ARG
    assert out.value is None


@needs_lib
def test_build_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = _lib.load()
    out = ctypes.c_void_p()
    off = np.array([0, 4], np.int64)
    rc = lib.tsk_index_build(ctypes.c_void_p(0x1000), off.ctypes.data_as(ctypes.c_void_p), 1, 3,
                             None, None, ctypes.byref(out))
    assert rc == _lib.TSK_ERR_DEVICE
    assert out.value is None


@needs_lib
def test_query_rejects_null_index():
    lib = _lib.load()
    off = np.array([0, 4], np.int64)
    rc = lib.tsk_knn_query(None, ctypes.c_void_p(0x1000), off.ctypes.data_as(ctypes.c_void_p), 1, 5,
                           1, _lib.band_struct(None), None, ctypes.c_void_p(0x2000),
                           ctypes.c_void_p(0x3000), None, None)
    assert rc == _lib.TSK_ERR_INVALID_ARG
    assert lib.tsk_index_free(None) == 0


def test_binding_refuses_without_library(monkeypatch, tmp_path):
    import paper_1811_11076_amd._lib as L
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "lib_path", lambda: str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        L.load()


@needs_lib
def test_query_and_tune_reject_null_index():
    lib = _lib.load()
    off = np.array([0, 4], np.int64)
    offp = off.ctypes.data_as(ctypes.c_void_p)
    fake = ctypes.c_void_p(0x1000)
    band = _lib.band_struct(None)
    rc = lib.tsk_knn_query(None, fake, offp, 1, 3, _lib.TSK_DK, band, None, fake, fake, None, None)
    assert rc == _lib.TSK_ERR_INVALID_ARG and b"index is NULL" in lib.tsk_last_error()
    rc = lib.tsk_tune(None, fake, offp, 1, 3, _lib.TSK_DTW, band, None, None, None, None, None)
    assert rc == _lib.TSK_ERR_INVALID_ARG
    rc = lib.tsk_pair_distances(None, fake, offp, 1, _lib.TSK_DK, band, fake, None)
    assert rc == _lib.TSK_ERR_INVALID_ARG


@needs_lib
def test_model_shape_and_file_errors_before_device_work(tmp_path):
    lib = _lib.load()
    h = ctypes.c_void_p()
    size = ctypes.sizeof(_lib.MlpShape)
    for dim, points, hidden, embed, code in ((0, 32, 256, 64, _lib.TSK_ERR_UNSUPPORTED),
                                             (9, 32, 256, 64, _lib.TSK_ERR_UNSUPPORTED),
                                             (3, 1, 256, 64, _lib.TSK_ERR_UNSUPPORTED),
                                             (3, 32, 100, 64, _lib.TSK_ERR_UNSUPPORTED),
                                             (3, 32, 256, 300, _lib.TSK_ERR_UNSUPPORTED)):
        sh = _lib.MlpShape(size, dim, points, hidden, embed)
        assert lib.tsk_model_create(ctypes.byref(sh), 0, ctypes.byref(h)) == code
        assert h.value is None
    bad = _lib.MlpShape(size + 8, 3, 32, 256, 64)
    assert lib.tsk_model_create(ctypes.byref(bad), 0, ctypes.byref(h)) == _lib.TSK_ERR_INVALID_ARG
    assert lib.tsk_model_create(None, 0, ctypes.byref(h)) == _lib.TSK_ERR_INVALID_ARG
    # unreadable and malformed encoder files
    missing = str(tmp_path / "missing.bin").encode()
    assert lib.tsk_model_load(missing, ctypes.byref(h)) == _lib.TSK_ERR_IO
    junk = tmp_path / "junk.bin"
    junk.write_bytes(b"not an encoder file at all")
    assert lib.tsk_model_load(str(junk).encode(), ctypes.byref(h)) == _lib.TSK_ERR_IO
    assert lib.tsk_model_save(None, missing) == _lib.TSK_ERR_INVALID_ARG
    assert lib.tsk_model_free(None) == _lib.TSK_OK


@needs_lib
def test_subseq_rejects_bad_arguments_before_device_work():
    lib = _lib.load()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    soff = np.array([0, 5000], np.int64)  # long series are fine here
    qoff = np.array([0, 8], np.int64)
    sp, qp = soff.ctypes.data_as(ctypes.c_void_p), qoff.ctypes.data_as(ctypes.c_void_p)

    def call(ser=fake, so=sp, n=1, dim=3, qv=fake, qo=qp, nq=1, k=1, opts=None, ids=fake,
             dist=fake, end=fake):
        return lib.tsk_subseq_query(ser, so, n, dim, qv, qo, nq, k, opts, ids, dist, end, None,
                                    None, None)

    assert call(ser=None) == _lib.TSK_ERR_INVALID_ARG
    assert call(qv=None) == _lib.TSK_ERR_INVALID_ARG
    assert call(dim=0) == _lib.TSK_ERR_UNSUPPORTED
    assert call(dim=9) == _lib.TSK_ERR_UNSUPPORTED
    assert call(k=0) == _lib.TSK_ERR_INVALID_ARG
    assert call(k=65) == _lib.TSK_ERR_UNSUPPORTED
    assert call(ids=None) == _lib.TSK_ERR_INVALID_ARG
    assert call(end=None) == _lib.TSK_ERR_INVALID_ARG
    assert call(so=None) == _lib.TSK_ERR_INVALID_ARG
    assert call(n=0) == _lib.TSK_ERR_INVALID_ARG
    empty = np.array([0, 0], np.int64)
    assert call(so=empty.ctypes.data_as(ctypes.c_void_p)) == _lib.TSK_ERR_INVALID_ARG
    long_q = np.array([0, 1025], np.int64)
    assert call(qo=long_q.ctypes.data_as(ctypes.c_void_p)) == _lib.TSK_ERR_UNSUPPORTED
    assert b"1025 > 1024" in lib.tsk_last_error()
    bad = _lib.SubseqOpts(ctypes.sizeof(_lib.SubseqOpts) + 8, 0, 1, 0, 0)
    assert call(opts=ctypes.byref(bad)) == _lib.TSK_ERR_INVALID_ARG
    bad = _lib.SubseqOpts(ctypes.sizeof(_lib.SubseqOpts), -1, 1, 0, 0)
    assert call(opts=ctypes.byref(bad)) == _lib.TSK_ERR_INVALID_ARG
    bad = _lib.SubseqOpts(ctypes.sizeof(_lib.SubseqOpts), 0, 2, 0, 0)
    assert call(opts=ctypes.byref(bad)) == _lib.TSK_ERR_INVALID_ARG
    import torch
    if not torch.cuda.is_available():
        # valid arguments reach the device query, which fails without a GPU
        assert call() == _lib.TSK_ERR_DEVICE


@needs_lib
def test_validate_values_arguments():
    lib = _lib.load()
    bad = ctypes.c_int64(5)
    assert lib.tsk_validate_values(None, 0, ctypes.byref(bad), None) == _lib.TSK_OK
    assert bad.value == -1
    assert lib.tsk_validate_values(None, 3, ctypes.byref(bad), None) == _lib.TSK_ERR_INVALID_ARG
    assert lib.tsk_validate_values(ctypes.c_void_p(0x1000), -1, None, None) == _lib.TSK_ERR_INVALID_ARG


def test_binding_rejects_host_outputs(monkeypatch):
    """Index.knn refuses out tensors that are not on the queries' device
    before any library call (a kernel writing to a host address faults)."""
    import torch
    import paper_1811_11076_amd as P

    class FakeLib:
        def tsk_knn_query(self, *a):
            raise AssertionError("the library must not be called")

    idx = P.Index.__new__(P.Index)
    idx._lib = FakeLib()
    idx._h = ctypes.c_void_p()
    idx.n, idx.dim = 10, 3
    monkeypatch.setattr(P, "_values", lambda v, dim=None: v)
    q = torch.zeros((8, 3), dtype=torch.float32)
    out = (torch.empty((1, 4), dtype=torch.int64), torch.empty((1, 4), dtype=torch.float32))
    with pytest.raises(ValueError, match="CUDA device"):
        idx.knn(q, np.array([0, 8]), 4, "dk", out=out)
