"""ctypes binding of libchr.so (include/chr.h).

Argument marshalling only: every step of compression, reconstruction and
extraction runs in the library's HIP kernels.  PyTorch supplies device
memory and the HIP stream.  The library must be built (``build()`` in
``__graft_entry__`` or ``python -m paper_2408_05462_amd.build``); importing
this module without it raises, there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libchr.so")

CHR_OK, CHR_E_INVAL, CHR_E_ACCURACY, CHR_E_LEVEL = 0, -1, -2, -3
CHR_E_CORRUPT, CHR_E_CAPACITY, CHR_E_NOMEM, CHR_E_HIP = -4, -5, -6, -7
CHR_E_CANCELLED, CHR_PENDING = -8, 1
STATUS_NAMES = {0: "CHR_OK", -1: "CHR_E_INVAL", -2: "CHR_E_ACCURACY", -3: "CHR_E_LEVEL", -4: "CHR_E_CORRUPT",
                -5: "CHR_E_CAPACITY", -6: "CHR_E_NOMEM", -7: "CHR_E_HIP", -8: "CHR_E_CANCELLED", 1: "CHR_PENDING"}

EXPORTS = ["chr_last_error", "chr_version", "chr_compress_bound", "chr_compress_workspace", "chr_compress",
           "chr_stream_info", "chr_stream_verify", "chr_reconstruct_workspace", "chr_reconstruct",
           "iso_workspace", "iso_extract", "iso_cases", "chr_mc_table", "chr_range", "chr_prof_enable",
           "chr_prof_collect", "chr_prof_disable", "chr_set_tiles", "chr_set_level0_tiles", "chr_batch_create", "chr_batch_workspace",
           "chr_batch_run", "chr_batch_capture", "chr_batch_replay", "chr_batch_autotune", "chr_batch_tune", "chr_batch_config", "chr_batch_set_config",
           "chr_batch_destroy", "chr_server_create", "chr_server_add_stream", "chr_server_submit",
           "chr_server_step", "chr_server_poll", "chr_server_release", "chr_server_cancel", "chr_server_stats_get",
           "chr_server_now_ms", "chr_server_destroy", "chr_topology_workspace", "chr_topology_error_bound",
           "chr_reconstruct_range", "chr_entropy_bound", "chr_entropy_workspace", "chr_entropy_encode",
           "chr_entropy_info", "chr_entropy_decode", "chr_tiers_bound", "chr_tiers_workspace", "chr_tiers_compress",
           "chr_tiers_header", "chr_tiers_reconstruct_workspace", "chr_tiers_reconstruct", "chr_block_box",
           "iso_box_workspace", "iso_extract_box", "chr_reconstruct_static",
           "chr_reconstruct_bits", "iso_extract_bits"]


class ChrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class chr_params(C.Structure):
    _fields_ = [("levels", C.c_int), ("block", C.c_int), ("qmax", C.c_int), ("error_bound_far", C.c_double),
                ("merge", C.c_int)]


class chr_result(C.Structure):
    _fields_ = [("stream_bytes", C.c_uint64), ("n_outlier", C.c_uint64), ("n_corrected", C.c_uint64),
                ("status", C.c_int32), ("vmin", C.c_float), ("vmax", C.c_float), ("reserved", C.c_uint32)]


class chr_info(C.Structure):
    _fields_ = [("dims", C.c_int64 * 3), ("levels", C.c_int), ("block", C.c_int), ("qmax", C.c_int),
                ("n_iso", C.c_int), ("error_bound", C.c_double), ("inv", C.c_float), ("step", C.c_float),
                ("isovalues", C.c_float * 16), ("vmin", C.c_float), ("vmax", C.c_float),
                ("nblocks", C.c_int64), ("nb", C.c_int * 3), ("flags", C.c_uint32),
                ("total_bytes", C.c_uint64), ("n_outlier", C.c_uint64), ("n_corrected", C.c_uint64),
                ("payload_offset", C.c_uint64), ("error_bound_far", C.c_double), ("inv_far", C.c_float),
                ("step_far", C.c_float), ("merge", C.c_int), ("mb", C.c_int * 3)]


class chr_batch_item(C.Structure):
    _fields_ = [("d_field", C.c_void_p), ("dims", C.c_int64 * 3), ("error_bound", C.c_double), ("n_iso", C.c_int),
                ("isovalues", C.c_float * 16), ("params", chr_params), ("d_stream", C.c_void_p),
                ("stream_capacity", C.c_size_t), ("d_result", C.c_void_p), ("d_recon", C.c_void_p),
                ("d_vertices", C.c_void_p * 16), ("cap_v", C.c_int64 * 16), ("d_tris", C.c_void_p * 16),
                ("cap_t", C.c_int64 * 16), ("d_counts", C.c_void_p), ("d_status", C.c_void_p),
                ("spacing", C.c_float)]


class chr_server_config(C.Structure):
    _fields_ = [("slots", C.c_int), ("max_group", C.c_int), ("d_pool", C.c_void_p), ("pool_bytes", C.c_size_t)]


class chr_request_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("level", C.c_int32), ("dataset", C.c_int32), ("stream_index", C.c_int32),
                ("isovalue", C.c_float), ("group_size", C.c_int32), ("error_bound", C.c_double),
                ("n_vertices", C.c_int64), ("n_triangles", C.c_int64), ("d_vertices", C.c_void_p),
                ("d_triangles", C.c_void_p), ("t_submit_ms", C.c_double), ("t_admit_ms", C.c_double),
                ("t_done_ms", C.c_double)]


class chr_server_stats(C.Structure):
    _fields_ = [("queued", C.c_int64), ("in_flight", C.c_int64), ("done", C.c_int64), ("failed", C.c_int64),
                ("pool_used", C.c_size_t), ("pool_peak", C.c_size_t), ("groups", C.c_int64),
                ("grouped_requests", C.c_int64)]


MAX_TIERS = 8


class chr_tier_header(C.Structure):
    _fields_ = [("n_tiers", C.c_int), ("n_iso", C.c_int), ("dims", C.c_int64 * 3), ("levels", C.c_int),
                ("block", C.c_int), ("qmax", C.c_int), ("reserved", C.c_int), ("isovalues", C.c_float * 16),
                ("total_bytes", C.c_uint64), ("bound", C.c_double * MAX_TIERS),
                ("stream_offset", C.c_uint64 * MAX_TIERS), ("stream_bytes", C.c_uint64 * MAX_TIERS),
                ("n_corrections", C.c_uint64 * MAX_TIERS), ("index_offset", C.c_uint64 * MAX_TIERS),
                ("value_offset", C.c_uint64 * MAX_TIERS)]


RESULT_BYTES = C.sizeof(chr_result)

_lib = None


def load():
    """Loads libchr.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                          "(python -m paper_2408_05462_amd.build)")
    L = C.CDLL(LIB_PATH)
    i64p = C.POINTER(C.c_int64)
    vp = C.c_void_p
    L.chr_last_error.restype = C.c_char_p
    L.chr_version.restype = C.c_int
    L.chr_compress_bound.argtypes = [i64p, C.POINTER(chr_params)]
    L.chr_compress_bound.restype = C.c_size_t
    L.chr_compress_workspace.argtypes = [i64p, C.POINTER(chr_params)]
    L.chr_compress_workspace.restype = C.c_size_t
    L.chr_compress.argtypes = [vp, i64p, C.c_double, vp, C.c_int, C.POINTER(chr_params), vp, C.c_size_t, vp,
                               vp, vp, vp, C.c_size_t, vp]
    L.chr_compress.restype = C.c_int
    L.chr_stream_info.argtypes = [vp, C.c_size_t, C.POINTER(chr_info)]
    L.chr_stream_info.restype = C.c_int
    L.chr_stream_verify.argtypes = [vp, C.c_size_t]
    L.chr_stream_verify.restype = C.c_int
    L.chr_reconstruct_workspace.argtypes = [C.POINTER(chr_info), C.c_int]
    L.chr_reconstruct_workspace.restype = C.c_size_t
    L.chr_reconstruct.argtypes = [C.POINTER(chr_info), vp, C.c_size_t, C.c_int, C.c_double, vp, vp, vp,
                                  C.c_size_t, vp]
    L.chr_reconstruct.restype = C.c_int
    L.chr_reconstruct_static.argtypes = [C.POINTER(chr_info), vp, C.c_size_t, C.c_int, C.c_double, vp, vp, vp]
    L.chr_reconstruct_static.restype = C.c_int
    L.iso_workspace.argtypes = [i64p]
    L.iso_workspace.restype = C.c_size_t
    L.iso_extract.argtypes = [vp, i64p, C.c_float, C.c_float, vp, C.c_int64, vp, C.c_int64, vp, vp, C.c_size_t,
                              vp]
    L.iso_extract.restype = C.c_int
    L.chr_reconstruct_bits.argtypes = [C.POINTER(chr_info), vp, C.c_size_t, C.c_double, C.POINTER(C.c_float),
                                       C.c_int, vp, vp, vp, vp, C.c_size_t, vp]
    L.chr_reconstruct_bits.restype = C.c_int
    L.iso_extract_bits.argtypes = [vp, i64p, vp, C.c_float, C.c_float, vp, C.c_int64, vp, C.c_int64, vp, vp,
                                   C.c_size_t, vp]
    L.iso_extract_bits.restype = C.c_int
    L.iso_cases.argtypes = [vp, i64p, C.c_float, vp, vp, C.c_size_t, vp]
    L.iso_cases.restype = C.c_int
    L.chr_mc_table.argtypes = [vp, vp]
    L.chr_mc_table.restype = C.c_int
    L.chr_range.argtypes = [vp, C.c_int64, vp, vp]
    L.chr_range.restype = C.c_int
    L.chr_prof_enable.argtypes = [C.c_char_p, C.c_int]
    L.chr_prof_enable.restype = C.c_int
    L.chr_prof_collect.argtypes = [vp, C.c_int, C.POINTER(C.c_int)]
    L.chr_prof_collect.restype = C.c_int
    L.chr_prof_disable.restype = C.c_int
    L.chr_set_tiles.argtypes = [C.c_int, C.c_int]
    L.chr_set_tiles.restype = C.c_int
    L.chr_set_level0_tiles.argtypes = [C.c_int]
    L.chr_set_level0_tiles.restype = C.c_int
    L.chr_batch_create.argtypes = [C.POINTER(chr_batch_item), C.c_int, C.POINTER(vp)]
    L.chr_batch_create.restype = C.c_int
    L.chr_batch_workspace.argtypes = [vp]
    L.chr_batch_workspace.restype = C.c_size_t
    L.chr_batch_run.argtypes = [vp, vp, C.c_size_t, vp]
    L.chr_batch_run.restype = C.c_int
    L.chr_batch_capture.argtypes = [vp, vp, C.c_size_t, vp]
    L.chr_batch_capture.restype = C.c_int
    L.chr_batch_replay.argtypes = [vp, vp]
    L.chr_batch_replay.restype = C.c_int
    L.chr_batch_autotune.argtypes = [vp, vp, C.c_size_t, vp, C.c_char_p]
    L.chr_batch_autotune.restype = C.c_int
    L.chr_batch_tune.argtypes = [vp, vp, C.c_size_t, vp, C.c_char_p, C.POINTER(C.c_int)]
    L.chr_batch_tune.restype = C.c_int
    ip = C.POINTER(C.c_int)
    L.chr_batch_config.argtypes = [vp, ip, ip, ip, C.POINTER(C.c_float)]
    L.chr_batch_config.restype = C.c_int
    L.chr_batch_set_config.argtypes = [vp, C.c_int, C.c_int, C.c_int]
    L.chr_batch_set_config.restype = C.c_int
    L.chr_batch_destroy.argtypes = [vp]
    L.chr_batch_destroy.restype = C.c_int
    L.chr_server_create.argtypes = [C.POINTER(chr_server_config), C.POINTER(vp)]
    L.chr_server_create.restype = C.c_int
    L.chr_server_add_stream.argtypes = [vp, C.c_int, C.POINTER(chr_info), vp, C.c_size_t, ip]
    L.chr_server_add_stream.restype = C.c_int
    L.chr_server_submit.argtypes = [vp, C.c_int, C.c_float, C.c_double, C.c_int, C.POINTER(C.c_int64)]
    L.chr_server_submit.restype = C.c_int
    L.chr_server_step.argtypes = [vp, ip]
    L.chr_server_step.restype = C.c_int
    L.chr_server_poll.argtypes = [vp, C.c_int64, C.POINTER(chr_request_result)]
    L.chr_server_poll.restype = C.c_int
    L.chr_server_release.argtypes = [vp, C.c_int64]
    L.chr_server_release.restype = C.c_int
    L.chr_server_cancel.argtypes = [vp, C.c_int64]
    L.chr_server_cancel.restype = C.c_int
    L.chr_server_stats_get.argtypes = [vp, C.POINTER(chr_server_stats)]
    L.chr_server_stats_get.restype = C.c_int
    L.chr_server_now_ms.argtypes = [vp]
    L.chr_server_now_ms.restype = C.c_double
    L.chr_server_destroy.argtypes = [vp]
    L.chr_server_destroy.restype = C.c_int
    L.chr_reconstruct_range.argtypes = [C.POINTER(chr_info), vp, C.c_size_t, C.c_int, C.c_double, C.c_float,
                                        C.c_float, vp, vp, vp, C.c_size_t, vp]
    L.chr_reconstruct_range.restype = C.c_int
    L.chr_topology_workspace.restype = C.c_size_t
    L.chr_topology_error_bound.argtypes = [vp, i64p, vp, C.c_int, C.c_int64, vp, vp, C.c_size_t, vp]
    L.chr_topology_error_bound.restype = C.c_int
    L.chr_entropy_bound.argtypes = [C.c_uint64]
    L.chr_entropy_bound.restype = C.c_size_t
    L.chr_entropy_workspace.argtypes = [C.c_uint64]
    L.chr_entropy_workspace.restype = C.c_size_t
    L.chr_entropy_encode.argtypes = [vp, C.c_uint64, vp, C.c_size_t, vp, vp, C.c_size_t, vp]
    L.chr_entropy_encode.restype = C.c_int
    u64p = C.POINTER(C.c_uint64)
    L.chr_entropy_info.argtypes = [vp, C.c_size_t, u64p, u64p]
    L.chr_entropy_info.restype = C.c_int
    L.chr_entropy_decode.argtypes = [vp, vp, C.c_uint64, vp, C.c_uint64, vp, vp]
    L.chr_entropy_decode.restype = C.c_int
    L.chr_tiers_bound.argtypes = [i64p, C.c_int, C.POINTER(chr_params)]
    L.chr_tiers_bound.restype = C.c_size_t
    L.chr_tiers_workspace.argtypes = [i64p, C.POINTER(chr_params)]
    L.chr_tiers_workspace.restype = C.c_size_t
    L.chr_tiers_compress.argtypes = [vp, i64p, vp, C.c_int, vp, C.c_int, C.POINTER(chr_params), vp, C.c_size_t, vp,
                                     vp, C.c_size_t, vp]
    L.chr_tiers_compress.restype = C.c_int
    L.chr_tiers_header.argtypes = [vp, C.c_size_t, C.POINTER(chr_tier_header)]
    L.chr_tiers_header.restype = C.c_int
    L.chr_tiers_reconstruct_workspace.argtypes = [C.POINTER(chr_tier_header)]
    L.chr_tiers_reconstruct_workspace.restype = C.c_size_t
    L.chr_tiers_reconstruct.argtypes = [C.POINTER(chr_tier_header), vp, C.c_size_t, C.c_double, vp, vp, vp,
                                        C.c_size_t, C.POINTER(C.c_int), vp]
    L.chr_tiers_reconstruct.restype = C.c_int
    L.chr_block_box.argtypes = [vp, C.c_size_t, C.c_float, C.c_float, i64p, i64p, C.POINTER(C.c_int)]
    L.chr_block_box.restype = C.c_int
    L.iso_box_workspace.argtypes = [i64p]
    L.iso_box_workspace.restype = C.c_size_t
    L.iso_extract_box.argtypes = [vp, i64p, i64p, i64p, C.c_float, C.c_float, vp, C.c_int64, vp, C.c_int64, vp, vp,
                                  C.c_size_t, vp]
    L.iso_extract_box.restype = C.c_int
    _lib = L
    return L


def check(rc, what):
    if rc != CHR_OK:
        raise ChrError(rc, f"{what}: {load().chr_last_error().decode()}")


def dims3(shape):
    return (C.c_int64 * 3)(*[int(s) for s in shape])
