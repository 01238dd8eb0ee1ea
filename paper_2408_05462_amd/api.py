"""Torch-facing wrappers of the C ABI, with the same names as include/chr.h.

Each function marshals tensors into the C call; the work runs in the HIP
kernels of libchr.so.  Calls are asynchronous on the current (or given) HIP
stream unless noted.  ``compress``/``reconstruct``/``extract`` are
synchronous conveniences that also read back device-side status.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _s(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _need_cuda_f32(t, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")


def params(levels=3, block=64, qmax=32767, error_bound_far=0.0, merge=0):
    """error_bound_far > 0: differentiated error control; merge > 1: block
    merging before compression, at most `merge` blocks per axis of a unit
    (include/chr.h)."""
    return L.chr_params(levels, block, qmax, float(error_bound_far), int(merge))


# ------------------------------------------------------------------ compress

def chr_compress_bound(shape, p):
    n = L.load().chr_compress_bound(L.dims3(shape), C.byref(p))
    if n == 0:
        L.check(L.CHR_E_INVAL, "chr_compress_bound")
    return n


def chr_compress_workspace(shape, p):
    n = L.load().chr_compress_workspace(L.dims3(shape), C.byref(p))
    if n == 0:
        L.check(L.CHR_E_INVAL, "chr_compress_workspace")
    return n


def chr_compress(field, error_bound, isovalues, p, out, result, ws, codes=None, flags=None, stream=None):
    """Launches compression of `field` into the uint8 buffer `out`; `result`
    is a uint8 device buffer of at least RESULT_BYTES bytes."""
    _need_cuda_f32(field, "field")
    iso = np.ascontiguousarray(np.asarray(isovalues, np.float32).reshape(-1))
    rc = L.load().chr_compress(_p(field), L.dims3(field.shape), float(error_bound), iso.ctypes.data_as(C.c_void_p),
                               len(iso), C.byref(p), _p(out), out.numel(), _p(result), _p(codes), _p(flags), _p(ws),
                               ws.numel(), _s(stream))
    L.check(rc, "chr_compress")


def read_result(result):
    r = L.chr_result.from_buffer_copy(bytes(result[: L.RESULT_BYTES].cpu().numpy()))
    return dict(stream_bytes=int(r.stream_bytes), n_outlier=int(r.n_outlier), n_corrected=int(r.n_corrected),
                status=int(r.status), vmin=float(r.vmin), vmax=float(r.vmax))


@dataclass
class Compressed:
    stream: torch.Tensor      # uint8 on the device, exactly stream_bytes long
    info: L.chr_info          # parsed header
    header: bytes             # host copy of header + tables
    result: dict


def compress(field, error_bound, isovalues=(), levels=3, block=64, qmax=32767, codes=None, flags=None,
             error_bound_far=0.0, merge=0):
    """Synchronous compression; raises ChrError on any device-side status."""
    p = params(levels, block, qmax, error_bound_far, merge)
    dev = field.device
    cap = chr_compress_bound(field.shape, p)
    out = torch.empty(cap, dtype=torch.uint8, device=dev)
    res = torch.zeros(64, dtype=torch.uint8, device=dev)
    ws = torch.empty(chr_compress_workspace(field.shape, p), dtype=torch.uint8, device=dev)
    chr_compress(field, error_bound, isovalues, p, out, res, ws, codes, flags)
    torch.cuda.synchronize(dev)
    r = read_result(res)
    if r["status"] != 0:
        raise L.ChrError(r["status"], "chr_compress (device status)")
    s = out[: r["stream_bytes"]]
    info, head = chr_stream_info_dev(s)
    return Compressed(stream=s, info=info, header=head, result=r)


# ------------------------------------------------------------------ stream inspection

def chr_stream_info(host_bytes):
    buf = np.ascontiguousarray(np.frombuffer(bytes(host_bytes), np.uint8))
    info = L.chr_info()
    rc = L.load().chr_stream_info(buf.ctypes.data_as(C.c_void_p), buf.size, C.byref(info))
    L.check(rc, "chr_stream_info")
    return info


def chr_stream_info_dev(stream_dev):
    """Copies the header and tables of a device stream to the host and parses them."""
    head = bytes(stream_dev[:256].cpu().numpy())
    info = chr_stream_info(head)
    head = bytes(stream_dev[: int(info.payload_offset)].cpu().numpy())
    info = chr_stream_info(head)
    return info, head


def chr_stream_verify(host_bytes):
    buf = np.ascontiguousarray(np.frombuffer(bytes(host_bytes), np.uint8))
    return L.load().chr_stream_verify(buf.ctypes.data_as(C.c_void_p), buf.size)


# ------------------------------------------------------------------ reconstruct

def stream_bound(info):
    """The bound a stream guarantees at every point (its far bound under
    differentiated error control)."""
    return info.error_bound_far if info.flags & 2 else info.error_bound


def level_shape(info, level):
    return tuple(((int(n) - 1) >> level) + 1 for n in info.dims)


def chr_reconstruct_workspace(info, level):
    n = L.load().chr_reconstruct_workspace(C.byref(info), level)
    if n == 0:
        L.check(L.CHR_E_LEVEL, "chr_reconstruct_workspace")
    return n


def chr_reconstruct(info, stream_dev, level, error_bound, out, status, ws, stream=None):
    rc = L.load().chr_reconstruct(C.byref(info), _p(stream_dev), stream_dev.numel(), level, float(error_bound),
                                  _p(out), _p(status), _p(ws), 0 if ws is None else ws.numel(), _s(stream))
    L.check(rc, "chr_reconstruct")


def chr_reconstruct_static(info, stream_dev, level, error_bound, out, status, stream=None):
    """chr_reconstruct with the coarser-level grids in the library's static
    device array (no workspace argument, no allocation)."""
    rc = L.load().chr_reconstruct_static(C.byref(info), _p(stream_dev), stream_dev.numel(), level,
                                         float(error_bound), _p(out), _p(status), _s(stream))
    L.check(rc, "chr_reconstruct_static")


def chr_reconstruct_range(info, stream_dev, level, error_bound, kmin, kmax, out, status, ws, stream=None):
    rc = L.load().chr_reconstruct_range(C.byref(info), _p(stream_dev), stream_dev.numel(), level, float(error_bound),
                                        float(np.float32(kmin)), float(np.float32(kmax)), _p(out), _p(status), _p(ws),
                                        0 if ws is None else ws.numel(), _s(stream))
    L.check(rc, "chr_reconstruct_range")


def reconstruct_range(c: Compressed, kmin, kmax, level=0):
    """Synchronous restricted reconstruction (see chr_reconstruct_range)."""
    dev = c.stream.device
    out = torch.empty(level_shape(c.info, level), dtype=torch.float32, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    ws = torch.empty(max(chr_reconstruct_workspace(c.info, level), 256), dtype=torch.uint8, device=dev)
    chr_reconstruct_range(c.info, c.stream, level, stream_bound(c.info), kmin, kmax, out, status, ws)
    torch.cuda.synchronize(dev)
    st = int(status.item())
    if st != 0:
        raise L.ChrError(st, "chr_reconstruct_range (device status)")
    return out


def reconstruct(c: Compressed, level=0, error_bound=None):
    eb = stream_bound(c.info) if error_bound is None else error_bound
    dev = c.stream.device
    out = torch.empty(level_shape(c.info, level), dtype=torch.float32, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    ws = torch.empty(max(chr_reconstruct_workspace(c.info, level), 256), dtype=torch.uint8, device=dev)
    chr_reconstruct(c.info, c.stream, level, eb, out, status, ws)
    torch.cuda.synchronize(dev)
    st = int(status.item())
    if st != 0:
        raise L.ChrError(st, "chr_reconstruct (device status)")
    return out


# ------------------------------------------------------------------ extract

def iso_workspace(shape):
    n = L.load().iso_workspace(L.dims3(shape))
    if n == 0:
        L.check(L.CHR_E_INVAL, "iso_workspace")
    return n


def iso_extract(field, isovalue, spacing, verts, tris, counts, ws, stream=None):
    _need_cuda_f32(field, "field")
    rc = L.load().iso_extract(_p(field), L.dims3(field.shape), float(np.float32(isovalue)), float(spacing),
                              _p(verts), 0 if verts is None else verts.shape[0], _p(tris),
                              0 if tris is None else tris.shape[0], _p(counts), _p(ws), ws.numel(), _s(stream))
    L.check(rc, "iso_extract")


def bits_shape(dims, n_iso=1):
    """Shape of n_iso planes of classification bits (uint64 words) for a field of dims."""
    return (n_iso, int(dims[0]) * int(dims[1]) * ((int(dims[2]) + 63) // 64))


def chr_reconstruct_bits(info, stream_dev, error_bound, isovalues, out, bits, status, ws, stream=None):
    ks = (C.c_float * len(isovalues))(*[float(np.float32(k)) for k in isovalues])
    rc = L.load().chr_reconstruct_bits(C.byref(info), _p(stream_dev), stream_dev.numel(), float(error_bound), ks,
                                       len(isovalues), _p(out), _p(bits), _p(status), _p(ws),
                                       0 if ws is None else ws.numel(), _s(stream))
    L.check(rc, "chr_reconstruct_bits")


def iso_extract_bits(field, bits_plane, isovalue, spacing, verts, tris, counts, ws, stream=None):
    _need_cuda_f32(field, "field")
    rc = L.load().iso_extract_bits(_p(field), L.dims3(field.shape), _p(bits_plane), float(np.float32(isovalue)),
                                   float(spacing), _p(verts), 0 if verts is None else verts.shape[0], _p(tris),
                                   0 if tris is None else tris.shape[0], _p(counts), _p(ws), ws.numel(), _s(stream))
    L.check(rc, "iso_extract_bits")


def reconstruct_bits(c, isovalues):
    """Synchronous level-0 reconstruction with the classification bits of
    each isovalue: (field, bits [n_iso, words] as int64)."""
    dev = c.stream.device
    out = torch.empty(level_shape(c.info, 0), dtype=torch.float32, device=dev)
    bits = torch.empty(bits_shape(out.shape, len(isovalues)), dtype=torch.int64, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    ws = torch.empty(max(chr_reconstruct_workspace(c.info, 0), 256), dtype=torch.uint8, device=dev)
    chr_reconstruct_bits(c.info, c.stream, stream_bound(c.info), isovalues, out, bits, status, ws)
    torch.cuda.synchronize(dev)
    st = int(status.item())
    if st != 0:
        raise L.ChrError(st, "chr_reconstruct_bits (device status)")
    return out, bits


def extract_bits(field, bits_plane, isovalue, spacing=1.0):
    """Synchronous marching cubes from given classification bits."""
    dev = field.device
    ws = torch.empty(iso_workspace(field.shape), dtype=torch.uint8, device=dev)
    counts = torch.zeros(2, dtype=torch.int64, device=dev)
    iso_extract_bits(field, bits_plane, isovalue, spacing, None, None, counts, ws)
    torch.cuda.synchronize(dev)
    nv, nt = (int(v) for v in counts.cpu())
    verts = torch.empty((max(nv, 1), 3), dtype=torch.float32, device=dev)
    tris = torch.empty((max(nt, 1), 3), dtype=torch.int32, device=dev)
    iso_extract_bits(field, bits_plane, isovalue, spacing, verts, tris, counts, ws)
    torch.cuda.synchronize(dev)
    return verts[:nv], tris[:nt]


def extract(field, isovalue, spacing=1.0):
    """Synchronous marching cubes: returns (verts [V,3] f32, tris [T,3] i32)."""
    dev = field.device
    ws = torch.empty(iso_workspace(field.shape), dtype=torch.uint8, device=dev)
    counts = torch.zeros(2, dtype=torch.int64, device=dev)
    iso_extract(field, isovalue, spacing, None, None, counts, ws)
    torch.cuda.synchronize(dev)
    nv, nt = (int(v) for v in counts.cpu())
    verts = torch.empty((max(nv, 1), 3), dtype=torch.float32, device=dev)
    tris = torch.empty((max(nt, 1), 3), dtype=torch.int32, device=dev)
    iso_extract(field, isovalue, spacing, verts, tris, counts, ws)
    torch.cuda.synchronize(dev)
    return verts[:nv], tris[:nt]


def iso_cases(field, isovalue, out, ws, stream=None):
    rc = L.load().iso_cases(_p(field), L.dims3(field.shape), float(np.float32(isovalue)), _p(out), _p(ws),
                            ws.numel(), _s(stream))
    L.check(rc, "iso_cases")


def cases(field, isovalue):
    dev = field.device
    cd = tuple(max(int(n) - 1, 0) for n in field.shape)
    out = torch.zeros(cd, dtype=torch.uint8, device=dev)
    ws = torch.empty(iso_workspace(field.shape), dtype=torch.uint8, device=dev)
    if min(cd) > 0:
        iso_cases(field, isovalue, out, ws)
        torch.cuda.synchronize(dev)
    return out


def chr_mc_table():
    ntri = np.zeros(256, np.uint8)
    tri = np.zeros((256, 15), np.int8)
    rc = L.load().chr_mc_table(ntri.ctypes.data_as(C.c_void_p), tri.ctypes.data_as(C.c_void_p))
    L.check(rc, "chr_mc_table")
    return ntri, tri


def chr_range(field, out, stream=None):
    rc = L.load().chr_range(_p(field), field.numel(), _p(out), _s(stream))
    L.check(rc, "chr_range")


def field_range(field):
    out = torch.zeros(4, dtype=torch.float32, device=field.device)
    chr_range(field, out)
    torch.cuda.synchronize(field.device)
    v = out.cpu()
    return float(v[0]), float(v[1]), int(v[2:3].view(torch.int32).item())


# ------------------------------------------------------------------ tiles and batches

def chr_set_tiles(enc_chunks_per_wave=8, dec_chunks_per_wave=16):
    L.check(L.load().chr_set_tiles(int(enc_chunks_per_wave), int(dec_chunks_per_wave)), "chr_set_tiles")


def chr_set_level0_tiles(on=True):
    L.check(L.load().chr_set_level0_tiles(1 if on else 0), "chr_set_level0_tiles")


class Batch:
    """Device buffers of a batch plus its chr_batch handle.

    fields: list of float32 CUDA tensors (any shapes); error_bounds and
    isovalues (a list per field, at most 16) and params (chr_params) per
    field.  mesh_caps[i][j] = (cap_v, cap_t) for field i, isovalue j; with
    mesh_caps=None the capacities are found by one eager run with no mesh
    outputs (the counts are written regardless), then the batch is planned
    again with buffers of exactly that size.
    """

    def __init__(self, fields, error_bounds, isovalues, params_list, spacing=1.0, mesh_caps=None, stream=None):
        self.fields = fields
        self.error_bounds = [float(e) for e in error_bounds]
        self.isovalues = [[float(np.float32(k)) for k in ks] for ks in isovalues]
        self.params = params_list
        self.spacing = float(spacing)
        dev = fields[0].device
        self.streams = [torch.empty(chr_compress_bound(f.shape, p), dtype=torch.uint8, device=dev)
                        for f, p in zip(fields, params_list)]
        self.results = [torch.zeros(64, dtype=torch.uint8, device=dev) for _ in fields]
        self.recon = [torch.empty_like(f) for f in fields]
        self.counts = [torch.zeros((max(len(k), 1), 2), dtype=torch.int64, device=dev) for k in self.isovalues]
        self.status = [torch.zeros(1, dtype=torch.int32, device=dev) for _ in fields]
        self.handle = None
        self.ws = None
        if mesh_caps is None:
            self._plan([[(0, 0)] * len(k) for k in self.isovalues])
            self.run(stream)
            torch.cuda.synchronize(dev)
            mesh_caps = [[(int(c[j, 0]), int(c[j, 1])) for j in range(len(k))]
                         for c, k in zip((c.cpu().numpy() for c in self.counts), self.isovalues)]
        self._plan(mesh_caps)

    def _plan(self, mesh_caps):
        dev = self.fields[0].device
        self.verts = [[torch.empty((max(cv, 1), 3), dtype=torch.float32, device=dev) for cv, _ in mc]
                      for mc in mesh_caps]
        self.tris = [[torch.empty((max(ct, 1), 3), dtype=torch.int32, device=dev) for _, ct in mc]
                     for mc in mesh_caps]
        items = (L.chr_batch_item * len(self.fields))()
        for i, f in enumerate(self.fields):
            _need_cuda_f32(f, "field")
            it = items[i]
            it.d_field = f.data_ptr()
            for a in range(3):
                it.dims[a] = int(f.shape[a])
            it.error_bound = self.error_bounds[i]
            it.n_iso = len(self.isovalues[i])
            for j, k in enumerate(self.isovalues[i]):
                it.isovalues[j] = k
                it.d_vertices[j] = self.verts[i][j].data_ptr()
                it.cap_v[j] = mesh_caps[i][j][0]
                it.d_tris[j] = self.tris[i][j].data_ptr()
                it.cap_t[j] = mesh_caps[i][j][1]
            it.params = self.params[i]
            it.d_stream = self.streams[i].data_ptr()
            it.stream_capacity = self.streams[i].numel()
            it.d_result = self.results[i].data_ptr()
            it.d_recon = self.recon[i].data_ptr()
            it.d_counts = self.counts[i].data_ptr()
            it.d_status = self.status[i].data_ptr()
            it.spacing = self.spacing
        self.close()
        h = C.c_void_p()
        L.check(L.load().chr_batch_create(items, len(self.fields), C.byref(h)), "chr_batch_create")
        self.handle = h
        nws = L.load().chr_batch_workspace(h)
        if self.ws is None or self.ws.numel() < nws:
            self.ws = torch.empty(nws, dtype=torch.uint8, device=dev)

    def run(self, stream=None):
        L.check(L.load().chr_batch_run(self.handle, _p(self.ws), self.ws.numel(), _s(stream)), "chr_batch_run")

    def capture(self, stream=None):
        L.check(L.load().chr_batch_capture(self.handle, _p(self.ws), self.ws.numel(), _s(stream)),
                "chr_batch_capture")

    def replay(self, stream=None):
        L.check(L.load().chr_batch_replay(self.handle, _s(stream)), "chr_batch_replay")

    def autotune(self, cache_path=None, stream=None):
        L.check(L.load().chr_batch_autotune(self.handle, _p(self.ws), self.ws.numel(), _s(stream),
                                            None if cache_path is None else str(cache_path).encode()),
                "chr_batch_autotune")

    def tune(self, cache_path=None, stream=None):
        """Eager-timed search over brick size, branches and tiles, then one
        capture (chr_batch_tune); returns the chosen brick size (0: each
        item's own)."""
        blk = C.c_int(0)
        L.check(L.load().chr_batch_tune(self.handle, _p(self.ws), self.ws.numel(), _s(stream),
                                        None if cache_path is None else str(cache_path).encode(), C.byref(blk)),
                "chr_batch_tune")
        return int(blk.value)

    def set_config(self, branches, enc_cpw=8, dec_cpw=16):
        L.check(L.load().chr_batch_set_config(self.handle, int(branches), int(enc_cpw), int(dec_cpw)),
                "chr_batch_set_config")

    def config(self):
        b, e, d, ms = C.c_int(), C.c_int(), C.c_int(), C.c_float()
        L.check(L.load().chr_batch_config(self.handle, C.byref(b), C.byref(e), C.byref(d), C.byref(ms)),
                "chr_batch_config")
        return dict(branches=b.value, enc_cpw=e.value, dec_cpw=d.value, last_ms=ms.value)

    def outputs(self, i):
        """Host copies of item i: (stream bytes, result, reconstruction, [(verts, tris)...], status)."""
        r = read_result(self.results[i])
        c = self.counts[i].cpu().numpy()
        meshes = [(self.verts[i][j][: int(c[j, 0])].cpu().numpy(), self.tris[i][j][: int(c[j, 1])].cpu().numpy())
                  for j in range(len(self.isovalues[i]))]
        return (bytes(self.streams[i][: r["stream_bytes"]].cpu().numpy()), r, self.recon[i].cpu().numpy(), meshes,
                int(self.status[i].item()))

    def close(self):
        if self.handle is not None:
            L.load().chr_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ serving

class Server:
    """Request loop over resident streams (chr_server_*).  `pool` is a uint8
    device tensor the server allocates reconstructions, counting state and
    meshes from; the caller keeps the registered streams alive."""

    def __init__(self, pool, slots=4, max_group=8):
        self.pool = pool
        cfg = L.chr_server_config(int(slots), int(max_group), pool.data_ptr() if pool is not None else None,
                                  0 if pool is None else pool.numel())
        h = C.c_void_p()
        L.check(L.load().chr_server_create(C.byref(cfg), C.byref(h)), "chr_server_create")
        self.handle = h
        self._streams = []

    def add_stream(self, dataset, info, stream_dev):
        idx = C.c_int()
        L.check(L.load().chr_server_add_stream(self.handle, int(dataset), C.byref(info), _p(stream_dev),
                                               stream_dev.numel(), C.byref(idx)), "chr_server_add_stream")
        self._streams.append(stream_dev)
        return idx.value

    def submit(self, dataset, isovalue, accuracy, level=0):
        rid = C.c_int64()
        L.check(L.load().chr_server_submit(self.handle, int(dataset), float(np.float32(isovalue)), float(accuracy),
                                           int(level), C.byref(rid)), "chr_server_submit")
        return rid.value

    def step(self):
        n = C.c_int()
        L.check(L.load().chr_server_step(self.handle, C.byref(n)), "chr_server_step")
        return n.value

    def poll(self, rid):
        r = L.chr_request_result()
        L.check(L.load().chr_server_poll(self.handle, int(rid), C.byref(r)), "chr_server_poll")
        return r

    def mesh(self, rid):
        """Host copies (verts [V,3] f32, tris [T,3] i32) of a finished request."""
        r = self.poll(rid)
        if r.status != 0:
            raise L.ChrError(r.status, f"request {rid}")
        nv, nt = int(r.n_vertices), int(r.n_triangles)
        base = self.pool.data_ptr()
        v = self.pool[r.d_vertices - base: r.d_vertices - base + 12 * nv] if nv else self.pool[:0]
        t = self.pool[r.d_triangles - base: r.d_triangles - base + 12 * nt] if nt else self.pool[:0]
        return (v.view(torch.float32).reshape(nv, 3).cpu().numpy(), t.view(torch.int32).reshape(nt, 3).cpu().numpy())

    def release(self, rid):
        L.check(L.load().chr_server_release(self.handle, int(rid)), "chr_server_release")

    def cancel(self, rid):
        L.check(L.load().chr_server_cancel(self.handle, int(rid)), "chr_server_cancel")

    def stats(self):
        st = L.chr_server_stats()
        L.check(L.load().chr_server_stats_get(self.handle, C.byref(st)), "chr_server_stats_get")
        return {f: getattr(st, f) for f, _ in L.chr_server_stats._fields_}

    def now_ms(self):
        return L.load().chr_server_now_ms(self.handle)

    def drain(self, ids=None, timeout_s=120.0):
        """Steps until every request (or those in `ids`) has finished."""
        import time

        t_end = time.monotonic() + timeout_s
        while True:
            self.step()
            if ids is None:
                st = self.stats()
                if st["queued"] == 0 and st["in_flight"] == 0:
                    return
            elif all(self.poll(i).status != L.CHR_PENDING for i in ids):
                return
            if time.monotonic() > t_end:
                raise TimeoutError(f"server did not drain: {self.stats()}")

    def close(self):
        if getattr(self, "handle", None) is not None:
            L.load().chr_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ error translation

def chr_topology_error_bound(field, isovalues, nth, out, ws, stream=None):
    _need_cuda_f32(field, "field")
    iso = np.ascontiguousarray(np.asarray(isovalues, np.float32).reshape(-1))
    rc = L.load().chr_topology_error_bound(_p(field), L.dims3(field.shape), iso.ctypes.data_as(C.c_void_p), len(iso),
                                           int(nth), _p(out), _p(ws), ws.numel(), _s(stream))
    L.check(rc, "chr_topology_error_bound")


def topology_error_bound(field, isovalues, nth=1):
    """Synchronous: (bound, |D|) of the paper's error translation."""
    out = torch.zeros(2, dtype=torch.float64, device=field.device)
    ws = torch.empty(L.load().chr_topology_workspace(), dtype=torch.uint8, device=field.device)
    chr_topology_error_bound(field, isovalues, nth, out, ws)
    torch.cuda.synchronize(field.device)
    v = out.cpu().numpy()
    return float(v[0]), int(v[1])


# ------------------------------------------------------------------ entropy stage

def _need_cuda_u8(t, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.uint8 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous uint8 CUDA tensor")


def chr_entropy_bound(n):
    return int(L.load().chr_entropy_bound(int(n)))


def chr_entropy_workspace(n):
    return int(L.load().chr_entropy_workspace(int(n)))


def chr_entropy_encode(data, out, result, ws, stream=None):
    """Asynchronous; ``result`` (2 x uint64 on the device) receives the size and the status."""
    _need_cuda_u8(data, "data")
    _need_cuda_u8(out, "out")
    rc = L.load().chr_entropy_encode(_p(data), data.numel(), _p(out), out.numel(), _p(result), _p(ws), ws.numel(),
                                     _s(stream))
    L.check(rc, "chr_entropy_encode")


def chr_entropy_info(head):
    """(n, total bytes) from the first 64 bytes of an entropy-coded stream (host bytes)."""
    h = np.ascontiguousarray(np.frombuffer(bytes(head[:64]), np.uint8))
    n, total = C.c_uint64(), C.c_uint64()
    rc = L.load().chr_entropy_info(h.ctypes.data_as(C.c_void_p), h.size, C.byref(n), C.byref(total))
    L.check(rc, "chr_entropy_info")
    return int(n.value), int(total.value)


def chr_entropy_decode(head, enc, out, status, stream=None):
    """Asynchronous; ``status`` (one int32 on the device) becomes 0 or CHR_E_CORRUPT."""
    _need_cuda_u8(enc, "enc")
    _need_cuda_u8(out, "out")
    h = np.ascontiguousarray(np.frombuffer(bytes(head[:64]), np.uint8))
    rc = L.load().chr_entropy_decode(h.ctypes.data_as(C.c_void_p), _p(enc), enc.numel(), _p(out), out.numel(),
                                     _p(status), _s(stream))
    L.check(rc, "chr_entropy_decode")


def entropy_encode(data):
    """Synchronous: the entropy-coded bytes of a uint8 CUDA tensor, as a CUDA tensor."""
    n = data.numel()
    out = torch.empty(max(chr_entropy_bound(n), 8), dtype=torch.uint8, device=data.device)
    ws = torch.empty(chr_entropy_workspace(n), dtype=torch.uint8, device=data.device)
    res = torch.zeros(2, dtype=torch.int64, device=data.device)
    chr_entropy_encode(data, out, res, ws)
    torch.cuda.synchronize(data.device)
    size, st = (int(v) for v in res.cpu())
    if st:
        raise L.ChrError(st, "chr_entropy_encode: output beyond its capacity")
    return out[:size]


def entropy_decode(enc):
    """Synchronous: the bytes an entropy-coded CUDA tensor holds."""
    head = enc[:64].cpu().numpy()
    n, _ = chr_entropy_info(head)
    out = torch.empty(max(n, 8), dtype=torch.uint8, device=enc.device)
    status = torch.zeros(1, dtype=torch.int32, device=enc.device)
    chr_entropy_decode(head, enc, out, status)
    torch.cuda.synchronize(enc.device)
    st = int(status.item())
    if st:
        raise L.ChrError(st, "chr_entropy_decode: corrupt stream")
    return out[:n]


# ------------------------------------------------------------------ multi-tier progressive accuracy

def chr_tiers_bound(shape, n_tiers, p):
    n = L.load().chr_tiers_bound(L.dims3(shape), int(n_tiers), C.byref(p))
    if n == 0:
        L.check(L.CHR_E_INVAL, "chr_tiers_bound")
    return n


def chr_tiers_workspace(shape, p):
    n = L.load().chr_tiers_workspace(L.dims3(shape), C.byref(p))
    if n == 0:
        L.check(L.CHR_E_INVAL, "chr_tiers_workspace")
    return n


def chr_tiers_compress(field, bounds, isovalues, p, out, result, ws, stream=None):
    """Asynchronous; ``result`` (2 x uint64 on the device) receives the size and the status."""
    _need_cuda_f32(field, "field")
    b = np.ascontiguousarray(np.asarray(bounds, np.float64).reshape(-1))
    iso = np.ascontiguousarray(np.asarray(isovalues, np.float32).reshape(-1))
    rc = L.load().chr_tiers_compress(_p(field), L.dims3(field.shape), b.ctypes.data_as(C.c_void_p), len(b),
                                     iso.ctypes.data_as(C.c_void_p), len(iso), C.byref(p), _p(out), out.numel(),
                                     _p(result), _p(ws), ws.numel(), _s(stream))
    L.check(rc, "chr_tiers_compress")


def chr_tiers_header(head):
    h = np.ascontiguousarray(np.frombuffer(bytes(head[:640]), np.uint8))
    out = L.chr_tier_header()
    rc = L.load().chr_tiers_header(h.ctypes.data_as(C.c_void_p), h.size, C.byref(out))
    L.check(rc, "chr_tiers_header")
    return out


def chr_tiers_reconstruct(header, container, error_bound, out, status, ws, stream=None):
    """Asynchronous; returns the last tier decoded."""
    used = C.c_int(-1)
    rc = L.load().chr_tiers_reconstruct(C.byref(header), _p(container), container.numel(), float(error_bound),
                                        _p(out), _p(status), _p(ws), ws.numel(), C.byref(used), _s(stream))
    L.check(rc, "chr_tiers_reconstruct")
    return used.value


def tiers_compress(field, bounds, isovalues=(), levels=3, block=64, qmax=32767):
    """Synchronous: (container as a uint8 CUDA tensor, parsed header)."""
    p = params(levels, block, qmax)
    dev = field.device
    out = torch.empty(chr_tiers_bound(field.shape, len(bounds), p), dtype=torch.uint8, device=dev)
    ws = torch.empty(chr_tiers_workspace(field.shape, p), dtype=torch.uint8, device=dev)
    res = torch.zeros(2, dtype=torch.int64, device=dev)
    chr_tiers_compress(field, bounds, isovalues, p, out, res, ws)
    torch.cuda.synchronize(dev)
    size, st = (int(v) for v in res.cpu())
    if st:
        raise L.ChrError(st, "chr_tiers_compress (device status)")
    c = out[:size]
    return c, chr_tiers_header(c[:640].cpu().numpy())


def tiers_reconstruct(container, header, error_bound):
    """Synchronous: (field, last tier decoded)."""
    dev = container.device
    shape = tuple(int(v) for v in header.dims)
    out = torch.empty(shape, dtype=torch.float32, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    ws = torch.empty(L.load().chr_tiers_reconstruct_workspace(C.byref(header)), dtype=torch.uint8, device=dev)
    used = chr_tiers_reconstruct(header, container, error_bound, out, status, ws)
    torch.cuda.synchronize(dev)
    st = int(status.item())
    if st:
        raise L.ChrError(st, "chr_tiers_reconstruct (device status)")
    return out, used


# ------------------------------------------------------------------ block merging for extraction

def chr_block_box(head, kmin, kmax):
    """(lo, hi) of the merged box of the blocks that can hold an isosurface at
    some k in [kmin, kmax] (head: header and tables on the host), or None."""
    h = np.ascontiguousarray(np.frombuffer(bytes(head), np.uint8))
    lo, hi, found = (C.c_int64 * 3)(), (C.c_int64 * 3)(), C.c_int()
    rc = L.load().chr_block_box(h.ctypes.data_as(C.c_void_p), h.size, float(kmin), float(kmax), lo, hi,
                                C.byref(found))
    L.check(rc, "chr_block_box")
    return (tuple(lo), tuple(hi)) if found.value else None


def iso_box_workspace(box_shape):
    n = L.load().iso_box_workspace(L.dims3(box_shape))
    if n == 0:
        L.check(L.CHR_E_INVAL, "iso_box_workspace")
    return n


def iso_extract_box(field, lo, hi, isovalue, spacing, verts, tris, counts, ws, stream=None):
    _need_cuda_f32(field, "field")
    lo3, hi3 = L.dims3(lo), L.dims3(hi)
    rc = L.load().iso_extract_box(_p(field), L.dims3(field.shape), lo3, hi3, float(isovalue), float(spacing),
                                  _p(verts), 0 if verts is None else verts.shape[0], _p(tris),
                                  0 if tris is None else tris.shape[0], _p(counts), _p(ws), ws.numel(), _s(stream))
    L.check(rc, "iso_extract_box")


def extract_box(field, lo, hi, isovalue, spacing=1.0):
    """Synchronous marching cubes over the box lo..hi: (verts [V,3], tris [T,3])."""
    dev = field.device
    bd = tuple(h - l + 1 for l, h in zip(lo, hi))
    ws = torch.empty(iso_box_workspace(bd), dtype=torch.uint8, device=dev)
    counts = torch.zeros(2, dtype=torch.int64, device=dev)
    iso_extract_box(field, lo, hi, isovalue, spacing, None, None, counts, ws)
    torch.cuda.synchronize(dev)
    nv, nt = (int(v) for v in counts.cpu())
    verts = torch.empty((max(nv, 1), 3), dtype=torch.float32, device=dev)
    tris = torch.empty((max(nt, 1), 3), dtype=torch.int32, device=dev)
    iso_extract_box(field, lo, hi, isovalue, spacing, verts, tris, counts, ws)
    torch.cuda.synchronize(dev)
    return verts[:nv], tris[:nt]
