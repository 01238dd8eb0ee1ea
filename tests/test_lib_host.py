"""Host-side checks of the HIP library (no GPU needed): it loads, exports every
symbol include/chr.h declares, and its host-only calls agree with the oracle."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
from paper_2408_05462_amd import _lib as L
from paper_2408_05462_amd import api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "chr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(chr_\w+|iso_\w+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = L.load()
    names = _declared()
    assert "chr_compress" in names and "chr_reconstruct" in names and "iso_extract" in names
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(names) == sorted(L.EXPORTS)


def test_table_matches_oracle():
    ntri, tri = api.chr_mc_table()
    ontri, otri = oracle.mc_table()
    assert np.array_equal(ntri, ontri)
    for c in range(256):
        assert list(tri[c][: 3 * ntri[c]]) == list(otri[c][: 3 * ntri[c]])
        assert all(v == -1 for v in tri[c][3 * ntri[c]:])


@pytest.mark.parametrize("shape,nL,B", [((64, 64, 64), 3, 64), ((17, 30, 9), 3, 4), ((256, 256, 256), 5, 64),
                                        ((97, 65, 130), 4, 32), ((1, 1, 5), 2, 2)])
def test_compress_bound_matches_oracle(shape, nL, B):
    assert api.chr_compress_bound(shape, api.params(nL, B)) == oracle.compress_bound(shape, nL, B)


def test_invalid_params_rejected():
    with pytest.raises(L.ChrError):
        api.chr_compress_bound((10, 10, 10), api.params(3, 6))     # block not a multiple of 4
    with pytest.raises(L.ChrError):
        api.chr_compress_bound((0, 10, 10), api.params(3, 8))
    with pytest.raises(L.ChrError):
        api.chr_compress_bound((10, 10, 10), api.params(3, 8, qmax=40000))


def test_stream_info_and_verify_on_oracle_stream():
    f = np.random.default_rng(4).standard_normal((13, 17, 19)).astype(np.float32)
    r = oracle.compress(f, 0.05, [0.3, -0.2], levels=3, block=8)
    s = bytes(r["stream"])
    info = api.chr_stream_info(s)
    oinfo = oracle.stream_info(r["stream"])
    assert tuple(info.dims) == tuple(oinfo.dims) == f.shape
    assert (info.levels, info.block, info.n_iso) == (3, 8, 2)
    assert info.total_bytes == len(s) and info.payload_offset == oinfo.payload_offset
    assert info.n_outlier == oinfo.n_outlier and info.n_corrected == oinfo.n_corrected
    assert api.chr_stream_verify(s) == L.CHR_OK
    t = bytearray(s)
    t[len(s) // 2] ^= 1
    assert api.chr_stream_verify(bytes(t)) == L.CHR_E_CORRUPT
    t = bytearray(s)
    t[20] ^= 1
    with pytest.raises(L.ChrError):
        api.chr_stream_info(bytes(t))


def test_workspace_queries():
    p = api.params(5, 64)
    assert api.chr_compress_workspace((256, 256, 256), p) > 0
    f = np.zeros((33, 20, 70), np.float32)
    r = oracle.compress(f, 0.1, [], levels=2, block=16)
    info = api.chr_stream_info(bytes(r["stream"]))
    assert L.load().chr_reconstruct_workspace(C.byref(info), 0) > 0
    assert L.load().chr_reconstruct_workspace(C.byref(info), 2) == 0      # level outside the hierarchy
    assert api.iso_workspace((33, 20, 70)) > 0
