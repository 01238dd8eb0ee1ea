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


@pytest.mark.parametrize("name", ["chr_batch_item", "chr_server_config", "chr_request_result",
                                  "chr_server_stats", "chr_info", "chr_result", "chr_params", "chr_tier_header"])
def test_struct_layout_matches_c(tmp_path, name):
    """Each ctypes mirror of a chr.h struct has the C compiler's layout."""
    import shutil
    import subprocess

    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("gcc not available")
    st = getattr(L, name)
    fields = [f for f, _ in st._fields_]
    src = tmp_path / "lay.c"
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "chr.h"\nint main(void){\n'
                   f'  printf("%zu\\n", sizeof({name}));\n'
                   + "".join(f'  printf("%zu\\n", offsetof({name}, {f}));\n' for f in fields) + "  return 0;\n}\n")
    exe = tmp_path / "lay"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    want = [C.sizeof(st)] + [getattr(st, f).offset for f in fields]
    assert got == want


def test_set_tiles_validates():
    lib = L.load()
    for e, d in [(0, 16), (3, 16), (32, 16), (4, 4), (4, 128), (4, 12)]:
        assert lib.chr_set_tiles(e, d) == L.CHR_E_INVAL
    for e in (1, 2, 4, 8, 16):
        for d in (8, 16, 32, 64):
            assert lib.chr_set_tiles(e, d) == L.CHR_OK
    assert lib.chr_set_tiles(8, 16) == L.CHR_OK  # the defaults


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
    assert 1 <= b.value <= len(shapes) and (e.value, d.value) == (8, 16)  # the process-wide tiles
    # manual configuration: validated, applied whole or not at all
    for bad_cfg in [(0, 8, 16), (len(shapes) + 1, 8, 16), (1, 3, 16), (1, 8, 12)]:
        assert lib.chr_batch_set_config(h, *bad_cfg) == L.CHR_E_INVAL
    assert lib.chr_batch_config(h, C.byref(b), C.byref(e), C.byref(d), C.byref(ms)) == L.CHR_OK
    assert (e.value, d.value) == (8, 16)
    assert lib.chr_batch_set_config(h, 1, 2, 32) == L.CHR_OK
    assert lib.chr_batch_config(h, C.byref(b), C.byref(e), C.byref(d), C.byref(ms)) == L.CHR_OK
    assert (b.value, e.value, d.value) == (1, 2, 32)
    # a replay before any capture is an error, not a launch
    assert lib.chr_batch_replay(h, None) == L.CHR_E_INVAL
    # the replay-timed autotuner is switched off: refused before any device call
    assert lib.chr_batch_autotune(h, 0x100000, 1 << 40, None, None) == L.CHR_E_INVAL
    assert b"switched off" in lib.chr_last_error()
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


def _tier_infos():
    """Host-parsed headers of oracle streams of one small field at three error bounds."""
    from paper_2408_05462_amd import inputs

    f = inputs.gaussians(24)
    out = []
    for rel in (1e-2, 1e-3, 1e-4):
        e = inputs.abs_error_bound(rel, f)
        ref = oracle.compress(f, e, [0.3, 0.5], levels=3, block=8)
        out.append((e, api.chr_stream_info(ref["stream"].tobytes()), ref["stream"].size))
    return out


def _server(pool_bytes=1 << 30, slots=2, group=4):
    lib = L.load()
    cfg = L.chr_server_config(slots, group, 0x100000, pool_bytes)  # placeholder address: never dereferenced here
    h = C.c_void_p()
    assert lib.chr_server_create(C.byref(cfg), C.byref(h)) == L.CHR_OK
    return lib, h


def test_server_config_validation():
    lib = L.load()
    h = C.c_void_p()
    for slots, group, pool, nbytes in [(0, 4, 0x1000, 1 << 20), (17, 4, 0x1000, 1 << 20), (2, 0, 0x1000, 1 << 20),
                                       (2, 65, 0x1000, 1 << 20), (2, 4, None, 1 << 20), (2, 4, 0x1000, 16)]:
        cfg = L.chr_server_config(slots, group, pool, nbytes)
        assert lib.chr_server_create(C.byref(cfg), C.byref(h)) == L.CHR_E_INVAL


def test_server_submit_selects_tier_and_rejects():
    """Submission is host logic: tier choice, and every rejection, happen
    before any device work (no GPU is touched here)."""
    tiers = _tier_infos()
    lib, h = _server()
    idx = C.c_int()
    for e, info, n in tiers:
        assert lib.chr_server_add_stream(h, 7, C.byref(info), 0x200000, n, C.byref(idx)) == L.CHR_OK
    # a stream shorter than its header states is refused
    assert lib.chr_server_add_stream(h, 8, C.byref(tiers[0][1]), 0x200000, 100, C.byref(idx)) == L.CHR_E_CORRUPT
    rid = C.c_int64()
    r = L.chr_request_result()
    # the loosest stream whose bound meets the accuracy serves the request
    for acc, want in [(tiers[0][0], 0), (tiers[0][0] * 0.99, 1), (tiers[1][0], 1), (1e9, 0), (tiers[2][0], 2)]:
        assert lib.chr_server_submit(h, 7, 0.4, acc, 0, C.byref(rid)) == L.CHR_OK
        assert lib.chr_server_poll(h, rid.value, C.byref(r)) == L.CHR_OK
        assert r.status == L.CHR_PENDING and r.stream_index == want and r.error_bound == tiers[want][0]
    n_ok = rid.value + 1
    assert lib.chr_server_submit(h, 7, 0.4, tiers[2][0] * 0.5, 0, C.byref(rid)) == L.CHR_E_ACCURACY
    assert lib.chr_server_submit(h, 9, 0.4, 1.0, 0, C.byref(rid)) == L.CHR_E_INVAL
    assert lib.chr_server_submit(h, 7, float("nan"), 1.0, 0, C.byref(rid)) == L.CHR_E_INVAL
    assert lib.chr_server_submit(h, 7, 0.4, 1.0, 3, C.byref(rid)) == L.CHR_E_LEVEL
    assert lib.chr_server_submit(h, 7, 0.4, 1.0, -1, C.byref(rid)) == L.CHR_E_LEVEL
    st = L.chr_server_stats()
    assert lib.chr_server_stats_get(h, C.byref(st)) == L.CHR_OK and st.queued == n_ok and st.in_flight == 0
    # cancel a queued request; release it; it is then unknown
    assert lib.chr_server_cancel(h, 1) == L.CHR_OK
    assert lib.chr_server_poll(h, 1, C.byref(r)) == L.CHR_OK and r.status == L.CHR_E_CANCELLED
    assert lib.chr_server_cancel(h, 1) == L.CHR_E_INVAL
    assert lib.chr_server_release(h, 0) == L.CHR_E_INVAL  # still queued
    assert lib.chr_server_release(h, 1) == L.CHR_OK
    assert lib.chr_server_poll(h, 1, C.byref(r)) == L.CHR_E_INVAL
    assert lib.chr_server_poll(h, 999, C.byref(r)) == L.CHR_E_INVAL
    assert lib.chr_server_stats_get(h, C.byref(st)) == L.CHR_OK and st.queued == n_ok - 1 and st.failed == 1
    assert lib.chr_server_destroy(h) == L.CHR_OK


def test_server_rejects_requests_larger_than_the_pool():
    tiers = _tier_infos()
    e, info, n = tiers[0]
    lib, h = _server(pool_bytes=64 << 10)
    idx = C.c_int()
    assert lib.chr_server_add_stream(h, 1, C.byref(info), 0x200000, n, C.byref(idx)) == L.CHR_OK
    rid = C.c_int64()
    # level 0 (24^3 reconstruction + counting state) exceeds 64 KiB; level 2 (6^3) fits
    assert lib.chr_server_submit(h, 1, 0.4, 1.0, 0, C.byref(rid)) == L.CHR_E_NOMEM
    assert lib.chr_server_submit(h, 1, 0.4, 1.0, 2, C.byref(rid)) == L.CHR_OK
    assert lib.chr_server_destroy(h) == L.CHR_OK


def test_topology_bound_rejects_bad_arguments():
    """Argument checks happen before any device work."""
    lib = L.load()
    ws_n = lib.chr_topology_workspace()
    assert 0 < ws_n < 1 << 16
    iso = (C.c_float * 2)(0.1, 0.2)
    fake = 0x100000
    dims = L.dims3((4, 5, 6))
    assert lib.chr_topology_error_bound(None, dims, iso, 2, 1, fake, fake, ws_n, None) == L.CHR_E_INVAL
    assert lib.chr_topology_error_bound(fake, L.dims3((0, 5, 6)), iso, 2, 1, fake, fake, ws_n, None) == L.CHR_E_INVAL
    assert lib.chr_topology_error_bound(fake, dims, iso, 17, 1, fake, fake, ws_n, None) == L.CHR_E_INVAL
    bad = (C.c_float * 1)(float("inf"))
    assert lib.chr_topology_error_bound(fake, dims, bad, 1, 1, fake, fake, ws_n, None) == L.CHR_E_INVAL
    assert lib.chr_topology_error_bound(fake, dims, iso, 2, 1, fake, fake, ws_n - 1, None) == L.CHR_E_NOMEM


def test_reciprocal_division_rule():
    """The level-0 kernels divide by block-shape constants d as trunc(fl(n * r))
    with r the smallest binary32 value >= 1/d; this equals floor(n / d) for
    n, d < 2^21 (checked for every n against small and sampled large d)."""
    n = np.arange(1 << 21, dtype=np.uint32)
    nf = n.astype(np.float32)
    rng = np.random.default_rng(3)
    ds = list(range(1, 200)) + [int(v) for v in rng.integers(200, 1 << 21, 60)] + [(1 << 21) - 1]
    for d in ds:
        r = np.float32(1.0 / d)
        if float(r) < 1.0 / d:
            r = np.nextafter(r, np.float32(np.inf))
        q = (nf * r).astype(np.uint32)
        assert np.array_equal(q, n // np.uint32(d)), d


@pytest.mark.parametrize("n", [0, 1, 511, 512, 513, 70000, 10**9])
def test_entropy_bound_matches_oracle(n):
    assert api.chr_entropy_bound(n) == oracle.entropy_bound(n)
    assert api.chr_entropy_workspace(n) >= 2304 + 8 * (n // 512)   # table, chunk sizes


def test_entropy_info_reads_oracle_headers_and_rejects_others():
    d = np.random.default_rng(3).integers(0, 9, 1234).astype(np.uint8)
    enc = oracle.entropy_encode(d)
    assert api.chr_entropy_info(enc[:64]) == (1234, enc.size)
    bad = enc[:64].copy()
    bad[0] ^= 1                                        # magic
    with pytest.raises(L.ChrError):
        api.chr_entropy_info(bad)
    bad = enc[:64].copy()
    bad[17] = 4                                        # chunk size 512 -> 1024
    with pytest.raises(L.ChrError):
        api.chr_entropy_info(bad)
    bad = enc[:64].copy()
    bad[20] += 1                                       # chunk count inconsistent with n
    with pytest.raises(L.ChrError):
        api.chr_entropy_info(bad)
    with pytest.raises(L.ChrError):
        api.chr_entropy_info(enc[:40])                 # short header


def test_entropy_calls_reject_bad_arguments_on_the_host():
    lib = L.load()
    buf = (C.c_uint64 * 16)()
    p = C.cast(buf, C.c_void_p)
    odd = C.c_void_p(p.value + 1)
    ws = api.chr_entropy_workspace(100)
    assert lib.chr_entropy_encode(None, 100, p, 1000, p, p, ws, None) == L.CHR_E_INVAL
    assert lib.chr_entropy_encode(odd, 100, p, 1000, p, p, ws, None) == L.CHR_E_INVAL
    assert lib.chr_entropy_encode(p, 1 << 32, p, 1000, p, p, 1 << 40, None) == L.CHR_E_INVAL
    assert lib.chr_entropy_encode(p, 100, p, 1000, p, p, ws - 1, None) == L.CHR_E_NOMEM
    enc = oracle.entropy_encode(np.arange(100, dtype=np.uint8))
    h = np.ascontiguousarray(enc[:64])
    hp = h.ctypes.data_as(C.c_void_p)
    # size disagreeing with the header, output too small: rejected before any launch
    assert lib.chr_entropy_decode(hp, p, enc.size - 8, p, 100, p, None) == L.CHR_E_CORRUPT
    assert lib.chr_entropy_decode(hp, p, enc.size, p, 99, p, None) == L.CHR_E_CAPACITY
    assert lib.chr_entropy_decode(hp, None, enc.size, p, 100, p, None) == L.CHR_E_INVAL


def test_differentiated_stream_header_is_parsed():
    f = np.random.default_rng(6).standard_normal((13, 17, 19)).astype(np.float32)
    s = oracle.compress(f, 0.01, [2.0], levels=3, block=8, error_bound_far=0.25)["stream"]
    info = api.chr_stream_info(bytes(s))
    assert info.flags & 2 and info.error_bound_far == 0.25
    assert info.inv_far == np.float32(1 / 0.5) and info.step_far == np.float32(0.5)
    assert api.stream_bound(info) == 0.25
    assert lib_verify(bytes(s)) == L.CHR_OK
    u = oracle.compress(f, 0.01, [2.0], levels=3, block=8)["stream"]
    iu = api.chr_stream_info(bytes(u))
    assert not iu.flags & 2 and iu.error_bound_far == 0.0 and api.stream_bound(iu) == 0.01


def lib_verify(b):
    return L.load().chr_stream_verify(b, len(b))


def test_far_bound_rejected_on_the_host():
    lib = L.load()
    fake = C.c_void_p(0x100000)
    for far in (1e-4, float("inf"), float("nan"), -1.0):
        p = api.params(3, 8, error_bound_far=far)
        rc = lib.chr_compress(fake, L.dims3((20, 20, 20)), 1e-3, None, 0, C.byref(p), fake, 1 << 20, fake, None,
                              None, fake, 1 << 30, None)
        assert rc == L.CHR_E_INVAL, far
        items = _items([(20, 20, 20)])
        items[0].params = p
        h = C.c_void_p()
        assert lib.chr_batch_create(items, 1, C.byref(h)) == L.CHR_E_INVAL


def test_tier_header_parsed_from_oracle_container():
    f = np.random.default_rng(12).standard_normal((12, 13, 14)).astype(np.float32)
    c = oracle.tiers_compress(f, [0.1, 0.01, 0.0], [0.3], levels=3, block=8)
    h = api.chr_tiers_header(c[:640])
    assert h.n_tiers == 3 and h.n_iso == 1 and list(h.dims) == [12, 13, 14] and h.total_bytes == c.size
    assert list(h.bound)[:3] == [0.1, 0.01, 0.0]
    assert h.stream_offset[0] == 640 and h.n_corrections[0] == 0
    bad = c[:640].copy()
    bad[8] = 9                                           # 9 tiers
    with pytest.raises(L.ChrError):
        api.chr_tiers_header(bad)
    bad = c[:640].copy()
    bad[128:136] = np.frombuffer(np.float64(0.001).tobytes(), np.uint8)   # bounds no longer decreasing
    with pytest.raises(L.ChrError):
        api.chr_tiers_header(bad)
    assert api.chr_tiers_bound((12, 13, 14), 3, api.params(3, 8)) == oracle.tiers_bound((12, 13, 14), 3, 3, 8)


def test_tier_bounds_rejected_on_the_host():
    lib = L.load()
    fake = C.c_void_p(0x100000)
    p = api.params(3, 8)
    for bounds in ([0.01, 0.01], [0.01, 0.02], [-1.0], [float("nan")], [0.1 / 2 ** i for i in range(9)]):
        b = np.asarray(bounds, np.float64)
        rc = lib.chr_tiers_compress(fake, L.dims3((20, 20, 20)), b.ctypes.data_as(C.c_void_p), len(b), None, 0,
                                    C.byref(p), fake, 1 << 30, fake, fake, 1 << 40, None)
        assert rc == L.CHR_E_INVAL, bounds
    pf = api.params(3, 8, error_bound_far=0.5)
    b = np.asarray([0.1], np.float64)
    assert lib.chr_tiers_compress(fake, L.dims3((20, 20, 20)), b.ctypes.data_as(C.c_void_p), 1, None, 0, C.byref(pf),
                                  fake, 1 << 30, fake, fake, 1 << 40, None) == L.CHR_E_INVAL


def test_block_box_matches_oracle_on_the_host():
    z, y, x = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in (30, 31, 33)], indexing="ij")
    f = np.exp(-((z - 7) ** 2 + (y - 8) ** 2 + (x - 9) ** 2) / 18.0).astype(np.float32)
    s = oracle.compress(f, 1e-4, [0.5], levels=3, block=8)["stream"]
    info = oracle.stream_info(s)
    head = bytes(s[: info.payload_offset])
    for kmin, kmax in [(0.5, 0.5), (0.2, 0.9), (5.0, 6.0), (-1.0, 0.0)]:
        assert api.chr_block_box(head, kmin, kmax) == oracle.block_box(s, kmin, kmax), (kmin, kmax)
    with pytest.raises(L.ChrError):
        api.chr_block_box(head, 1.0, 0.5)
    with pytest.raises(L.ChrError):
        api.chr_block_box(head[:300], 0.5, 0.5)


def test_merged_stream_info_bound_and_rejections():
    """Merged streams (block merging before compression) from the oracle:
    the library's header parser reads the units and checks their tiling; the
    bound and the argument checks of merging."""
    import struct

    f = np.random.default_rng(8).standard_normal((21, 19, 23)).astype(np.float32)
    r = oracle.compress(f, 0.05, [], levels=2, block=4, merge=3)
    s = bytes(r["stream"])
    info = api.chr_stream_info(s)
    oinfo = oracle.stream_info(r["stream"])
    assert info.flags == 8 and info.merge == 3 and tuple(info.mb) == tuple(oinfo.mb)
    assert info.nblocks == oinfo.nblocks < 6 * 5 * 6
    assert info.payload_offset == oinfo.payload_offset
    assert api.chr_stream_verify(s) == L.CHR_OK
    # a box entry moved onto another unit: caught once the tables' checksum
    # is made consistent again
    t = bytearray(s)
    xt = info.payload_offset - 32 * info.nblocks
    t[xt + 32: xt + 44] = t[xt: xt + 12]
    words = np.frombuffer(bytes(t[256: info.payload_offset]), "<u4").astype(np.uint64)
    j = (np.arange(len(words), dtype=np.uint64) * np.uint64(0x9E3779B9)) & np.uint64(0xFFFFFFFF)
    h = words ^ j
    for sh, mul in ((16, 0x85EBCA6B), (13, 0xC2B2AE35)):
        h = ((h ^ (h >> np.uint64(sh))) * np.uint64(mul)) & np.uint64(0xFFFFFFFF)
    h ^= h >> np.uint64(16)
    t[248:252] = struct.pack("<I", int(h.sum() & np.uint64(0xFFFFFFFF)))
    hw = np.frombuffer(bytes(t[:252]), "<u4").astype(np.uint64)
    j = (np.arange(63, dtype=np.uint64) * np.uint64(0x9E3779B9)) & np.uint64(0xFFFFFFFF)
    h = hw ^ j
    for sh, mul in ((16, 0x85EBCA6B), (13, 0xC2B2AE35)):
        h = ((h ^ (h >> np.uint64(sh))) * np.uint64(mul)) & np.uint64(0xFFFFFFFF)
    h ^= h >> np.uint64(16)
    t[252:256] = struct.pack("<I", int(h.sum() & np.uint64(0xFFFFFFFF)))
    with pytest.raises(L.ChrError):
        api.chr_stream_info(bytes(t))
    api.chr_stream_info(bytes(t[:256]))     # the header alone does not hold the units
    # bound: the plain bound plus a box entry per block
    shape = (65, 70, 129)
    nb = 2 * 3 * 4
    assert (api.chr_compress_bound(shape, api.params(3, 32, merge=2))
            == api.chr_compress_bound(shape, api.params(3, 32)) + 32 * nb
            == oracle.compress_bound(shape, 3, 32) + 32 * nb)
    for dims, bad in (((40, 40, 40), api.params(3, 8, merge=17)), ((40, 40, 40), api.params(3, 8, merge=-1)),
                      ((40, 40, 40), api.params(3, 8, error_bound_far=1.0, merge=2)),
                      ((2049, 2049, 2049), api.params(1, 1024, merge=2))):   # units of 2049^3 points
        with pytest.raises(L.ChrError):
            api.chr_compress_bound(dims, bad)
    api.chr_compress_bound((2049, 2049, 2049), api.params(1, 1024))
    assert api.chr_compress_workspace((64, 64, 64), api.params(3, 16, merge=2)) > \
        api.chr_compress_workspace((64, 64, 64), api.params(3, 16))
