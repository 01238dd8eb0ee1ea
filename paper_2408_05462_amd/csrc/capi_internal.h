// capi_internal.h -- host-side planning shared by the single-field calls
// (capi.hip) and the batch runner (batch.hip).  Each *_prepare function
// validates its arguments, lays the workspace out and fills a launch plan;
// the caller then launches it on a stream of its choice.
#pragma once

#include <string>

#include "../../include/chr.h"
#include "chr_plan.h"

namespace chr {

// Sets the calling thread's chr_last_error() text; returns code.
int api_fail(int code, const std::string &msg);
// Turns a pending HIP launch error into CHR_E_HIP.
int api_check_launch(const char *what);

// The bound a stream guarantees at every point: its far bound under
// differentiated error control, its error bound otherwise.
inline double stream_bound(const chr_info &I) { return (I.flags & 2u) ? I.error_bound_far : I.error_bound; }

struct EncJob {
  EncPlan P;
  U4 *scan;
  uint64_t *scan64;
  uint32_t *units;   // merged units: box table and first slots (workspace)
  int64_t *ubase;
};

struct DecJob {
  DecPlan D;
};

struct McJob {
  McPlan M;
  U4 *scan;
};

size_t enc_workspace_bytes(const int64_t dims[3], const chr_params *p);
// merging: whether the caller runs enc_merge_units (block merging, p->merge > 1)
int enc_prepare(const float *d_field, const int64_t dims[3], double error_bound, const float *h_iso, int n_iso,
                const chr_params *p, void *d_stream, size_t capacity, chr_result *d_result, int32_t *d_codes,
                uint8_t *d_flags, void *d_ws, size_t ws_bytes, int cpw0, EncJob &J, bool merging = false);
// Block merging before compression: units from the blocks' signatures
// (waits for stream s once); the plan then covers units.
int enc_merge_units(EncJob &J, hipStream_t s);

// Reconstruction plan from the compression geometry (quantizer constants and
// isovalues already set), for streams whose header is not on the host.
size_t dec_workspace_bytes(const Geo &g, int level);
int dec_prepare(const Geo &g, uint64_t payload_off, int level, const void *d_stream, uint64_t stream_bytes,
                float *d_out, int32_t *d_status, void *d_ws, size_t ws_bytes, int cpw0, DecJob &J);

size_t mc_workspace_bytes(const int64_t dims[3]);
int mc_prepare(const float *d_field, const int64_t dims[3], float isovalue, float spacing, float *d_vertices,
               int64_t cap_v, int32_t *d_tris, int64_t cap_t, int64_t *d_counts, void *d_ws, size_t ws_bytes,
               McJob &J);

// Compression geometry of a field (no device pointers): block grid,
// quantizer constants, sorted distinct isovalues, stream table size.
int enc_geometry(const int64_t dims[3], double error_bound, const float *h_iso, int n_iso, const chr_params *p,
                 Geo &g, uint64_t &payload_off);

// Reconstruction of a parsed stream into d_out with the compact grids of the
// coarser levels in d_ws (ws_bytes); krange (optional, 2 floats) restricts it
// to the blocks an isovalue range needs.  Every chr_reconstruct* entry point
// ends here.
int reconstruct_impl(const chr_info *info, const void *d_stream, size_t stream_bytes, int level, double error_bound,
                     const float *krange, float *d_out, int32_t *d_status, void *d_ws, size_t ws_bytes, void *stream);
// Bytes of coarser-level grids a reconstruction to `level` needs (0 when the
// header or level is invalid, or when nothing is needed).
size_t reconstruct_need(const chr_info *info, int level);

bool tiles_ok(int enc_cpw, int dec_cpw);
// The process-wide level-0 tiles (chr_set_tiles).
void current_tiles(int &enc_cpw, int &dec_cpw);

// Geometry of a stream from its parsed header (parameters, quantizer
// constants and lossless flag checked against each other).
int info_geo(const chr_info *I, Geo &g);

}  // namespace chr
