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


def test_batch_item_layout_matches_c(tmp_path):
    """The ctypes mirror of chr_batch_item has the C compiler's layout."""
    import shutil
    import subprocess

    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("gcc not available")
    fields = [f for f, _ in L.chr_batch_item._fields_]
    src = tmp_path / "lay.c"
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "chr.h"\nint main(void){\n'
                   '  printf("%zu\\n", sizeof(chr_batch_item));\n'
                   + "".join(f'  printf("%zu\\n", offsetof(chr_batch_item, {f}));\n' for f in fields) + "  return 0;\n}\n")
    exe = tmp_path / "lay"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    want = [C.sizeof(L.chr_batch_item)] + [getattr(L.chr_batch_item, f).offset for f in fields]
    assert got == want


def test_set_tiles_validates():
    lib = L.load()
    for e, d in [(0, 16), (3, 16), (32, 16), (4, 4), (4, 128), (4, 12)]:
        assert lib.chr_set_tiles(e, d) == L.CHR_E_INVAL
    for e in (1, 2, 4, 8, 16):
        for d in (8, 16, 32, 64):
            assert lib.chr_set_tiles(e, d) == L.CHR_OK
    assert lib.chr_set_tiles(4, 16) == L.CHR_OK


def _items(shapes, n_iso=2, fake=0x100000):
    """Batch items with placeholder device addresses (planning never touches them)."""
    items = (L.chr_batch_item * len(shapes))()
    for i, sh in enumerate(shapes):
        it = items[i]
        it.d_field = it.d_stream = it.d_result = it.d_recon = it.d_counts = fake
        for a in range(3):
            it.dims[a] = sh[a]
        it.error_bound = 1e-3
        it.n_iso = n_iso
        for j in range(n_iso):
            it.isovalues[j] = 0.1 * j
        it.params = api.params(3, 16)
        it.stream_capacity = api.chr_compress_bound(sh, it.params)
        it.spacing = 1.0
    return items


def test_batch_plan_workspace_and_rejections():
    lib = L.load()
    shapes = [(33, 40, 47), (64, 64, 64), (17, 23, 29)]
    items = _items(shapes)
    h = C.c_void_p()
    assert lib.chr_batch_create(items, len(shapes), C.byref(h)) == L.CHR_OK
    ws = lib.chr_batch_workspace(h)
    per = max(max(lib.chr_compress_workspace(L.dims3(s), C.byref(items[0].params)), lib.iso_workspace(L.dims3(s)))
              for s in shapes)
    assert ws >= len(shapes) * per
    assert ws <= len(shapes) * (per + 256 + 4 * 64 ** 3)
    b, e, d, ms = C.c_int(), C.c_int(), C.c_int(), C.c_float()
    assert lib.chr_batch_config(h, C.byref(b), C.byref(e), C.byref(d), C.byref(ms)) == L.CHR_OK
    assert 1 <= b.value <= len(shapes) and (e.value, d.value) == (4, 16)
    # a replay before any capture is an error, not a launch
    assert lib.chr_batch_replay(h, None) == L.CHR_E_INVAL
    assert lib.chr_batch_destroy(h) == L.CHR_OK

    bad = _items(shapes)
    bad[1].d_recon = None
    assert lib.chr_batch_create(bad, len(shapes), C.byref(h)) == L.CHR_E_INVAL
    assert b"item 1" in lib.chr_last_error()
    bad = _items(shapes)
    bad[2].stream_capacity = 100
    assert lib.chr_batch_create(bad, len(shapes), C.byref(h)) == L.CHR_E_CAPACITY
    bad = _items(shapes)
    bad[0].params = api.params(3, 6)  # block not a multiple of 2^(levels-1)
    assert lib.chr_batch_create(bad, len(shapes), C.byref(h)) == L.CHR_E_INVAL
    bad = _items(shapes)
    bad[0].n_iso = 17
    assert lib.chr_batch_create(bad, len(shapes), C.byref(h)) == L.CHR_E_INVAL
    bad = _items(shapes)
    bad[0].cap_v[0] = 10  # capacity without a buffer
    assert lib.chr_batch_create(bad, len(shapes), C.byref(h)) == L.CHR_E_INVAL
    assert lib.chr_batch_create(items, 0, C.byref(h)) == L.CHR_E_INVAL
