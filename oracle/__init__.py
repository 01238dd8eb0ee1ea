"""CPU oracle for the CHR hot path (test infrastructure only).

This package wraps ``chr_oracle.c``, the plain CPU reference that the GPU
library is checked against.  Only the test suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import it.  It shares no code with
the GPU library and never imports it.

Paper: "Accelerating In-transit Isosurface Generation With Topology Preserving
Compression" (arXiv 2408.05462), Sec. II.B (topology preservation, the edge
condition on d0/d1 and the error translation over D).  The hierarchy,
predictor, quantizer, stream format and triangle table are unspecified by the
paper; the readings implemented are documented in ``chr_oracle.c``.

Parity unpinned: compression ratio (the paper prints none).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "chr_oracle.c")
_SRC_ENT = os.path.join(_HERE, "chr_entropy.c")
_SRC_TIERS = os.path.join(_HERE, "chr_tiers.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, E_INVAL, E_ACCURACY, E_LEVEL, E_CORRUPT, E_CAPACITY, E_NOMEM = 0, -1, -2, -3, -4, -5, -6
MC_MAXTRI = 12


class OracleError(RuntimeError):
    def __init__(self, rc, what):
        super().__init__(f"{what}: oracle status {rc}")
        self.rc = rc


def build() -> str:
    """Compile the oracle (gcc, -O2 -ffp-contract=off, OpenMP)."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
           "-shared", "-std=c11", "-Wall", "-Wextra", _SRC, _SRC_ENT, _SRC_TIERS, "-o", _LIB + ".tmp",
           "-lm"]
    subprocess.check_call(cmd, cwd=_HERE)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or any(os.path.getmtime(f) > os.path.getmtime(_LIB)
                                           for f in (_SRC, _SRC_ENT, _SRC_TIERS, os.path.join(_HERE, "chr_oracle.h"))):
            build()
        L = C.CDLL(_LIB)
        i64p = C.POINTER(C.c_int64)
        L.orc_level_of.argtypes = [C.c_int64, C.c_int64, C.c_int64, C.c_int]
        L.orc_level_of.restype = C.c_int
        L.orc_predict.argtypes = [C.c_void_p, i64p, C.c_int64, C.c_int64, C.c_int64, C.c_int, C.c_int]
        L.orc_predict.restype = C.c_float
        L.orc_quantize.argtypes = [C.c_float, C.c_float, C.c_double, C.c_int, C.POINTER(C.c_int32),
                                   C.POINTER(C.c_int), C.POINTER(C.c_float)]
        L.orc_rank.argtypes = [C.c_float, C.c_void_p, C.c_int]
        L.orc_rank.restype = C.c_int
        L.orc_compress_bound.argtypes = [i64p, C.c_int, C.c_int]
        L.orc_compress_bound.restype = C.c_size_t
        L.orc_compress.argtypes = [C.c_void_p, i64p, C.c_double, C.c_double, C.c_void_p, C.c_int, C.c_int, C.c_int,
                                   C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                                   C.POINTER(C.c_size_t)]
        L.orc_compress.restype = C.c_int
        L.orc_compress_merged.argtypes = [C.c_void_p, i64p, C.c_double, C.c_double, C.c_void_p, C.c_int, C.c_int,
                                          C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                          C.c_size_t, C.POINTER(C.c_size_t)]
        L.orc_compress_merged.restype = C.c_int
        L.orc_compress_bound_merged.argtypes = [i64p, C.c_int, C.c_int, C.c_int]
        L.orc_compress_bound_merged.restype = C.c_size_t
        L.orc_stream_verify.argtypes = [C.c_void_p, C.c_size_t]
        L.orc_stream_codes.argtypes = [C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p]
        L.orc_decompress.argtypes = [C.c_void_p, C.c_size_t, C.c_int, C.c_double, C.c_void_p]
        L.orc_block_index.argtypes = [C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p]
        L.orc_mc_table.argtypes = [C.c_void_p, C.c_void_p]
        L.orc_mc_table.restype = None
        L.orc_mc_cases.argtypes = [C.c_void_p, i64p, C.c_float, C.c_void_p]
        L.orc_mc_cases.restype = None
        L.orc_mc.argtypes = [C.c_void_p, i64p, C.c_float, C.c_float, C.c_void_p, C.c_int64, C.c_void_p,
                             C.c_int64, i64p]
        L.orc_topology_error_bound.argtypes = [C.c_void_p, i64p, C.c_void_p, C.c_int, C.c_int64, i64p]
        L.orc_topology_error_bound.restype = C.c_double
        L.orc_stream_info.argtypes = [C.c_void_p, C.c_size_t, C.c_void_p]
        L.orc_threads.restype = C.c_int
        u64p = C.POINTER(C.c_uint64)
        L.orc_huff_lengths.argtypes = [C.c_void_p, C.c_int, C.c_void_p]
        L.orc_huff_codes.argtypes = [C.c_void_p, C.c_void_p]
        L.orc_entropy_bound.argtypes = [C.c_uint64, C.c_uint32, C.c_int]
        L.orc_entropy_bound.restype = C.c_uint64
        L.orc_entropy_encode.argtypes = [C.c_void_p, C.c_uint64, C.c_uint32, C.c_int, C.c_void_p, C.c_uint64, u64p]
        L.orc_entropy_info.argtypes = [C.c_void_p, C.c_uint64, u64p, C.POINTER(C.c_uint32)]
        L.orc_entropy_decode.argtypes = [C.c_void_p, C.c_uint64, C.c_void_p, C.c_uint64, u64p]
        _lib = L
    return _lib


def _dims(shape):
    return (C.c_int64 * 3)(*[int(s) for s in shape])


def _f32(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data


def threads():
    return lib().orc_threads()


def level_of(x, y, z, nL):
    return lib().orc_level_of(x, y, z, nL)


def predict(xr, x, y, z, level, nL):
    xr, p = _f32(xr)
    return float(lib().orc_predict(p, _dims(xr.shape), x, y, z, level, nL))


def quantize(x, p, e, qmax=32767):
    q, o, r = C.c_int32(), C.c_int(), C.c_float()
    lib().orc_quantize(x, p, e, qmax, C.byref(q), C.byref(o), C.byref(r))
    return q.value, o.value, np.float32(r.value)


def rank(v, iso):
    iso = np.ascontiguousarray(np.sort(np.asarray(iso, np.float32)))
    return lib().orc_rank(v, iso.ctypes.data, len(iso))


def compress_bound(shape, nL, block):
    return lib().orc_compress_bound(_dims(shape), nL, block)


def compress(x, error_bound, isovalues=(), levels=3, block=64, qmax=32767, error_bound_far=0.0, merge=0):
    """Returns dict(stream=bytes(np.uint8), q, flags, xr).  error_bound_far > 0
    selects differentiated error control (the far bound away from blocks that
    cross a candidate isovalue); merge > 1 merges blocks of equal index
    signature into units of at most `merge` blocks per axis before
    compression."""
    x, px = _f32(x)
    iso = np.ascontiguousarray(np.asarray(isovalues, np.float32).reshape(-1))
    cap = lib().orc_compress_bound_merged(_dims(x.shape), levels, block, int(merge))
    stream = np.zeros(cap, np.uint8)
    q = np.zeros(x.shape, np.int32)
    fl = np.zeros(x.shape, np.uint8)
    xr = np.zeros(x.shape, np.float32)
    nbytes = C.c_size_t()
    rc = lib().orc_compress_merged(px, _dims(x.shape), float(error_bound), float(error_bound_far), iso.ctypes.data,
                                   len(iso), levels, block, qmax, int(merge), q.ctypes.data, fl.ctypes.data,
                                   xr.ctypes.data, stream.ctypes.data, cap, C.byref(nbytes))
    if rc != OK:
        raise OracleError(rc, "orc_compress")
    return dict(stream=stream[: nbytes.value].copy(), q=q, flags=fl, xr=xr)


class Info(C.Structure):
    _fields_ = [("dims", C.c_int64 * 3), ("levels", C.c_int), ("block", C.c_int), ("qmax", C.c_int),
                ("n_iso", C.c_int), ("error_bound", C.c_double), ("inv", C.c_float), ("step", C.c_float),
                ("iso", C.c_float * 16), ("vmin", C.c_float), ("vmax", C.c_float), ("nblocks", C.c_int64),
                ("nb", C.c_int * 3), ("flags", C.c_uint32), ("total_bytes", C.c_uint64),
                ("n_outlier", C.c_uint64), ("n_corrected", C.c_uint64), ("payload_offset", C.c_uint64),
                ("error_bound_far", C.c_double), ("inv_far", C.c_float), ("step_far", C.c_float),
                ("merge", C.c_int), ("mb", C.c_int * 3)]


def stream_info(stream):
    s = np.ascontiguousarray(stream, np.uint8)
    info = Info()
    rc = lib().orc_stream_info(s.ctypes.data, s.size, C.byref(info))
    if rc != OK:
        raise OracleError(rc, "orc_stream_info")
    return info


def stream_verify(stream):
    s = np.ascontiguousarray(stream, np.uint8)
    return lib().orc_stream_verify(s.ctypes.data, s.size)


def stream_codes(stream):
    s = np.ascontiguousarray(stream, np.uint8)
    info = stream_info(s)
    shape = tuple(info.dims)
    q = np.zeros(shape, np.int32)
    e = np.zeros(shape, np.uint8)
    rc = lib().orc_stream_codes(s.ctypes.data, s.size, q.ctypes.data, e.ctypes.data)
    if rc != OK:
        raise OracleError(rc, "orc_stream_codes")
    return q, e


def decompress(stream, level=0, error_bound=None):
    s = np.ascontiguousarray(stream, np.uint8)
    info = stream_info(s)
    if error_bound is None:
        eb = info.error_bound_far if info.flags & 2 else info.error_bound
    else:
        eb = error_bound
    shape = tuple(((int(n) - 1) >> level) + 1 for n in info.dims)
    out = np.zeros(shape, np.float32)
    rc = lib().orc_decompress(s.ctypes.data, s.size, level, float(eb), out.ctypes.data)
    if rc != OK:
        raise OracleError(rc, "orc_decompress")
    return out


def decompress_rc(stream, level, error_bound):
    s = np.ascontiguousarray(stream, np.uint8)
    info = stream_info(s)
    shape = tuple(((int(n) - 1) >> max(level, 0)) + 1 for n in info.dims)
    out = np.zeros(shape, np.float32)
    return lib().orc_decompress(s.ctypes.data, s.size, level, float(error_bound), out.ctypes.data)


def block_index(stream):
    s = np.ascontiguousarray(stream, np.uint8)
    info = stream_info(s)
    mins = np.zeros(info.nblocks, np.float32)
    maxs = np.zeros(info.nblocks, np.float32)
    rc = lib().orc_block_index(s.ctypes.data, s.size, mins.ctypes.data, maxs.ctypes.data)
    if rc != OK:
        raise OracleError(rc, "orc_block_index")
    return mins, maxs


def mc_table():
    ntri = np.zeros(256, np.uint8)
    tri = np.zeros((256, 3 * MC_MAXTRI), np.int8)
    lib().orc_mc_table(ntri.ctypes.data, tri.ctypes.data)
    return ntri, tri


def mc_cases(f, k):
    f, pf = _f32(f)
    cd = tuple(max(int(n) - 1, 0) for n in f.shape)
    cases = np.zeros(cd, np.uint8)
    if min(cd) > 0:
        lib().orc_mc_cases(pf, _dims(f.shape), float(np.float32(k)), cases.ctypes.data)
    return cases


def mc(f, k, spacing=1.0, cap_v=None, cap_t=None):
    """Returns (verts [V,3] float32 xyz, tris [T,3] int32)."""
    f, pf = _f32(f)
    counts = (C.c_int64 * 2)()
    if cap_v is None or cap_t is None:
        rc = lib().orc_mc(pf, _dims(f.shape), float(np.float32(k)), float(spacing), None, 0, None, 0, counts)
        cap_v, cap_t = counts[0], counts[1]
    verts = np.zeros((max(cap_v, 1), 3), np.float32)
    tris = np.zeros((max(cap_t, 1), 3), np.int32)
    rc = lib().orc_mc(pf, _dims(f.shape), float(np.float32(k)), float(spacing), verts.ctypes.data, cap_v,
                      tris.ctypes.data, cap_t, counts)
    if rc not in (OK, E_CAPACITY):
        raise OracleError(rc, "orc_mc")
    return verts[: min(counts[0], cap_v)], tris[: min(counts[1], cap_t)], (counts[0], counts[1]), rc


def topology_error_bound(f, isovalues, nth=1):
    f, pf = _f32(f)
    iso = np.ascontiguousarray(np.asarray(isovalues, np.float32).reshape(-1))
    nd = C.c_int64()
    r = lib().orc_topology_error_bound(pf, _dims(f.shape), iso.ctypes.data, len(iso), nth, C.byref(nd))
    return r, nd.value


# ---- entropy stage (chr_entropy.c) ------------------------------------------
ENTROPY_CHUNK = 512
ENTROPY_MAXLEN = 12


def huff_lengths(hist, maxlen=ENTROPY_MAXLEN):
    """Code lengths of the 256 byte values from their counts."""
    h = np.ascontiguousarray(np.asarray(hist, np.uint64).reshape(256))
    out = np.zeros(256, np.uint8)
    rc = lib().orc_huff_lengths(h.ctypes.data, maxlen, out.ctypes.data)
    if rc:
        raise OracleError(rc, "huff_lengths")
    return out


def huff_codes(lengths):
    """Canonical codes (most significant bit first) of the lengths."""
    ln = np.ascontiguousarray(np.asarray(lengths, np.uint8).reshape(256))
    out = np.zeros(256, np.uint32)
    rc = lib().orc_huff_codes(ln.ctypes.data, out.ctypes.data)
    if rc:
        raise OracleError(rc, "huff_codes")
    return out


def entropy_bound(n, chunk=ENTROPY_CHUNK, maxlen=ENTROPY_MAXLEN):
    """Largest encoding of n bytes."""
    return int(lib().orc_entropy_bound(int(n), chunk, maxlen))


def entropy_encode(data, chunk=ENTROPY_CHUNK, maxlen=ENTROPY_MAXLEN):
    """The entropy stage's encoding of a byte string (uint8 array)."""
    d = np.ascontiguousarray(np.frombuffer(bytes(data), np.uint8) if not isinstance(data, np.ndarray) else data,
                             np.uint8)
    cap = int(lib().orc_entropy_bound(d.size, chunk, maxlen))
    out = np.zeros(max(cap, 1), np.uint8)
    nb = C.c_uint64()
    rc = lib().orc_entropy_encode(d.ctypes.data, d.size, chunk, maxlen, out.ctypes.data, cap, C.byref(nb))
    if rc:
        raise OracleError(rc, "entropy_encode")
    return out[: nb.value].copy()


def entropy_decode(enc):
    """Decodes an entropy-stage stream (uint8 array) back to its bytes."""
    e = np.ascontiguousarray(enc, np.uint8)
    n = C.c_uint64()
    ch = C.c_uint32()
    rc = lib().orc_entropy_info(e.ctypes.data, e.size, C.byref(n), C.byref(ch))
    if rc:
        raise OracleError(rc, "entropy_info")
    out = np.zeros(max(n.value, 1), np.uint8)
    rc = lib().orc_entropy_decode(e.ctypes.data, e.size, out.ctypes.data, n.value, C.byref(n))
    if rc:
        raise OracleError(rc, "entropy_decode")
    return out[: n.value].copy()


# ---- multi-tier progressive accuracy (chr_tiers.c) ---------------------------
MAX_TIERS = 8


def tiers_bound(shape, T, levels, block):
    L = lib()
    L.orc_tiers_bound.argtypes = [C.POINTER(C.c_int64), C.c_int, C.c_int, C.c_int]
    L.orc_tiers_bound.restype = C.c_uint64
    return int(L.orc_tiers_bound(_dims(shape), T, levels, block))


def tiers_compress(x, bounds, isovalues=(), levels=3, block=64, qmax=32767):
    """The tier container (uint8 array) of x at bounds[0] > bounds[1] > ..."""
    L = lib()
    x, px = _f32(x)
    b = np.ascontiguousarray(np.asarray(bounds, np.float64).reshape(-1))
    iso = np.ascontiguousarray(np.asarray(isovalues, np.float32).reshape(-1))
    cap = tiers_bound(x.shape, len(b), levels, block)
    out = np.zeros(cap, np.uint8)
    nb = C.c_uint64()
    L.orc_tiers_compress.argtypes = [C.c_void_p, C.POINTER(C.c_int64), C.c_void_p, C.c_int, C.c_void_p, C.c_int,
                                     C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_uint64, C.POINTER(C.c_uint64)]
    L.orc_tiers_compress.restype = C.c_int
    rc = L.orc_tiers_compress(px, _dims(x.shape), b.ctypes.data, len(b), iso.ctypes.data, len(iso), levels, block,
                              qmax, out.ctypes.data, cap, C.byref(nb))
    if rc:
        raise OracleError(rc, "tiers_compress")
    return out[: nb.value].copy()


def tiers_info(container):
    L = lib()
    c = np.ascontiguousarray(container, np.uint8)
    T = C.c_int()
    b = np.zeros(MAX_TIERS, np.float64)
    tot = C.c_uint64()
    L.orc_tiers_info.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(C.c_int), C.c_void_p, C.POINTER(C.c_uint64)]
    L.orc_tiers_info.restype = C.c_int
    rc = L.orc_tiers_info(c.ctypes.data, c.size, C.byref(T), b.ctypes.data, C.byref(tot))
    if rc:
        raise OracleError(rc, "tiers_info")
    return T.value, b[: T.value].copy(), tot.value


def tiers_decompress_rc(container, eb):
    """(status, field, last tier used)."""
    L = lib()
    c = np.ascontiguousarray(container, np.uint8)
    dims = tuple(int(v) for v in np.frombuffer(c[16:40].tobytes(), np.int64))
    out = np.zeros(dims, np.float32)
    used = C.c_int(-1)
    L.orc_tiers_decompress.argtypes = [C.c_void_p, C.c_uint64, C.c_double, C.c_void_p, C.POINTER(C.c_int)]
    L.orc_tiers_decompress.restype = C.c_int
    rc = L.orc_tiers_decompress(c.ctypes.data, c.size, float(eb), out.ctypes.data, C.byref(used))
    return rc, out, used.value


def tiers_decompress(container, eb):
    rc, out, used = tiers_decompress_rc(container, eb)
    if rc:
        raise OracleError(rc, "tiers_decompress")
    return out, used


# ---- block merging for extraction ----------------------------------------------

def block_box(stream, kmin, kmax):
    """(lo, hi) points (z, y, x; inclusive) of the merged box of the blocks
    that can hold a crossing of an isovalue in [kmin, kmax], or None."""
    L = lib()
    s = np.ascontiguousarray(stream, np.uint8)
    lo = (C.c_int64 * 3)()
    hi = (C.c_int64 * 3)()
    found = C.c_int()
    L.orc_block_box.argtypes = [C.c_void_p, C.c_size_t, C.c_float, C.c_float, C.c_void_p, C.c_void_p,
                                C.POINTER(C.c_int)]
    L.orc_block_box.restype = C.c_int
    rc = L.orc_block_box(s.ctypes.data, s.size, float(np.float32(kmin)), float(np.float32(kmax)), lo, hi,
                         C.byref(found))
    if rc:
        raise OracleError(rc, "block_box")
    return (tuple(lo), tuple(hi)) if found.value else None


def mc_box(f, lo, hi, k, spacing=1.0):
    """Marching cubes over the box lo..hi of f, with f's coordinates: (verts, tris)."""
    L = lib()
    f, pf = _f32(f)
    lo3 = (C.c_int64 * 3)(*lo)
    hi3 = (C.c_int64 * 3)(*hi)
    L.orc_mc_box.argtypes = [C.c_void_p, C.POINTER(C.c_int64), C.c_void_p, C.c_void_p, C.c_float, C.c_float,
                             C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p]
    L.orc_mc_box.restype = C.c_int
    counts = (C.c_int64 * 2)()
    rc = L.orc_mc_box(pf, _dims(f.shape), lo3, hi3, float(np.float32(k)), float(spacing), None, 0, None, 0, counts)
    cap_v, cap_t = counts[0], counts[1]
    verts = np.zeros((max(cap_v, 1), 3), np.float32)
    tris = np.zeros((max(cap_t, 1), 3), np.int32)
    rc = L.orc_mc_box(pf, _dims(f.shape), lo3, hi3, float(np.float32(k)), float(spacing), verts.ctypes.data, cap_v,
                      tris.ctypes.data, cap_t, counts)
    if rc not in (OK, E_CAPACITY):
        raise OracleError(rc, "mc_box")
    return verts[: counts[0]], tris[: counts[1]]
