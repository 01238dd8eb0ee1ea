/*
 * chr.h -- C ABI of the MI355X (gfx950) CHR library.
 *
 * Compressed Hierarchical Representation (CHR) with topology preservation for
 * 3D binary32 scalar fields, reconstruction at any hierarchy level, and
 * marching-cubes isosurface extraction, after "Accelerating In-transit
 * Isosurface Generation With Topology Preserving Compression" (arXiv
 * 2408.05462).  The data source compresses a field into a CHR; the
 * visualization side requests the data an isovalue needs at a given accuracy
 * and generates the isosurface (Sec. II, workflow description).
 *
 * Conventions for every call:
 *  - A field is float32 [nz][ny][nx], x fastest.  dims[] = {nz, ny, nx},
 *    each in [1, 2^30].
 *  - Pointers named d_* are device pointers (HIP global memory, gfx950);
 *    h_* are host pointers.  The caller owns every buffer it passes in;
 *    the library never frees caller memory and keeps no pointer after a call
 *    returns.
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *    Compute calls are asynchronous on that stream: the host-side return
 *    code reports argument errors only.  Conditions found on the device
 *    (non-finite input, too small an output buffer, a corrupt stream) are
 *    written to the device-side status/result words documented per call.
 *  - Workspace: every compute call takes a device scratch buffer d_ws of at
 *    least the size its *_workspace() query returns; the library allocates
 *    nothing on the device.
 *  - Return codes: CHR_OK or a negative CHR_E_* value; chr_last_error()
 *    returns a thread-local message for the last failure.
 */
#ifndef CHR_H
#define CHR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CHR_OK 0
#define CHR_E_INVAL (-1)    /* bad argument, or non-finite input value     */
#define CHR_E_ACCURACY (-2) /* requested error bound below the stream's     */
#define CHR_E_LEVEL (-3)    /* requested level not in the hierarchy         */
#define CHR_E_CORRUPT (-4)  /* stream fails its magic/version/checksums     */
#define CHR_E_CAPACITY (-5) /* output buffer too small; size reported       */
#define CHR_E_NOMEM (-6)    /* workspace too small                           */
#define CHR_E_HIP (-7)      /* a HIP runtime call failed                     */
#define CHR_E_CANCELLED (-8) /* served request cancelled before it finished  */
#define CHR_PENDING 1        /* served request still queued or in flight     */

/* Compression parameters.
 *  levels: nL, number of hierarchy levels (1..16).  Level nL-1 holds the
 *          anchors (points whose coordinates are all multiples of
 *          S = 2^(nL-1)); level l < nL-1 holds the points of the 2^l grid
 *          that are not on the 2^(l+1) grid.
 *  block:  B, edge of the cubic cell blocks of the domain decomposition
 *          (Sec. II.A: domain decomposition into blocks; Sec. III tests 64
 *          and 128).  Must be a multiple of S.  Each block stores the points
 *          of its closed extent [o, o+B] (faces shared with neighbours), so
 *          every block decodes on its own.  The closed extent must hold
 *          fewer than 2^31 points.
 *  qmax:   largest quantization code magnitude (1..32767). */
typedef struct chr_params {
  int levels;
  int block;
  int qmax;
  /* Differentiated error control (Sec. II.A, blocks with different error
   * bounds): 0 = error_bound everywhere; otherwise finite and >= error_bound,
   * the bound of every point that no block crossing a candidate isovalue
   * contains.  A block crosses isovalue k when min < k <= max over the input
   * on its closed extent; points of such blocks keep error_bound, so the
   * meshes of the candidate isovalues equal those of a stream compressed
   * with error_bound everywhere. */
  double error_bound_far;
  /* Block merging before compression (Sec. II.A, third step of CHR
   * generation: blocks merged into larger rectangular grids so that they are
   * compressed and visualized more efficiently).  0 or 1: none.  2..16: the
   * most blocks per axis of a merged unit.  A block's index signature is
   * the set of candidate isovalues its input crosses (min < k <= max over
   * its closed extent); blocks of equal signature are merged greedily in
   * lexicographic block order into rectangular units (grown along x, then y,
   * then z), each stored as one closed extent, so faces between merged
   * blocks are stored once.  Codes and reconstruction equal the unmerged
   * stream's; the block table then holds one record per unit and a box table
   * lists the units.  A unit's closed extent must hold fewer than 2^31
   * points; not combined with error_bound_far, batches or tier containers
   * (CHR_E_INVAL).  chr_compress with merging waits once for its stream
   * (the units are laid out on the host from the blocks' signatures). */
  int merge;
} chr_params;

/* Device-side result of chr_compress (caller-allocated device memory). */
typedef struct chr_result {
  uint64_t stream_bytes; /* bytes of the stream (the required size when status = CHR_E_CAPACITY) */
  uint64_t n_outlier;    /* points stored exactly because the bound or qmax failed */
  uint64_t n_corrected;  /* points stored exactly because their side of an isovalue changed */
  int32_t status;        /* CHR_OK, CHR_E_INVAL (non-finite input) or CHR_E_CAPACITY */
  float vmin, vmax;      /* range of the input field */
  uint32_t reserved;
} chr_result;

/* Parsed stream header (host side). */
typedef struct chr_info {
  int64_t dims[3];
  int levels, block, qmax, n_iso;
  double error_bound;
  float inv, step;       /* 1/(2e) and 2e as stored (binary32) */
  float isovalues[16];   /* sorted ascending, de-duplicated */
  float vmin, vmax;
  int64_t nblocks;
  int nb[3];
  uint32_t flags;        /* bit 0: lossless mode; bit 1: differentiated error control; bit 2: far quantizer
                            lossless; bit 3: merged units (nblocks then counts units) */
  uint64_t total_bytes, n_outlier, n_corrected, payload_offset;
  double error_bound_far;      /* flags bit 1: bound of points outside every active block (header bytes 192..199) */
  float inv_far, step_far;     /* its 1/(2e) and 2e (bytes 200..207) */
  int merge;                   /* flags bit 3: most blocks per axis of a unit (bytes 208..211); else 1 */
  int mb[3];                   /* largest unit extent in blocks along z, y, x (bytes 212..223); else 1 */
} chr_info;

const char *chr_last_error(void);
int chr_version(void);

/* ---- compression (Sec. II.A CHR generation; Sec. II.B topology
 *      preserving compression) ------------------------------------------ */

/* Upper bound on the stream size for these dims and parameters (every point
 * stored exactly).  0 on invalid arguments. */
size_t chr_compress_bound(const int64_t dims[3], const chr_params *p);

/* Workspace bytes chr_compress needs.  0 on invalid arguments. */
size_t chr_compress_workspace(const int64_t dims[3], const chr_params *p);

/* Compresses d_field into the CHR stream d_stream (capacity bytes).
 *
 * error_bound: absolute bound e >= 0 (finite); every reconstructed value x'
 *   satisfies |x' - x| <= e (checked in double).  e = 0 is lossless.
 * h_isovalues / n_iso: up to 16 candidate isovalues (host array; sorted and
 *   de-duplicated by the library).  For each of them every cell of the
 *   reconstructed field, at every level, keeps the marching-cubes case of
 *   the original field (Sec. II.B, topology preservation): a vertex whose
 *   reconstruction would change side of any candidate is stored exactly.
 * d_result: device chr_result, written when the work completes.
 * d_codes, d_flags: optional (may be NULL) per-point outputs in field layout:
 *   quantization code (0 where stored exactly) and flags (bit 0 outlier,
 *   bit 1 topology correction).
 * d_stream must be 8-byte aligned (CHR_E_INVAL otherwise).
 * Device-detected: non-finite input -> status CHR_E_INVAL (stream invalid);
 * stream larger than capacity -> status CHR_E_CAPACITY, stream_bytes = the
 * required size, nothing written beyond capacity (sections that do not fit
 * are not written at all). */
int chr_compress(const float *d_field, const int64_t dims[3], double error_bound,
                 const float *h_isovalues, int n_iso, const chr_params *p,
                 void *d_stream, size_t capacity, chr_result *d_result,
                 int32_t *d_codes, uint8_t *d_flags,
                 void *d_ws, size_t ws_bytes, void *stream);

/* ---- stream inspection (host) ------------------------------------------ */

/* Parses and validates a stream header from a host copy of its first n
 * bytes (n >= 256; if n also covers the section and block tables, their
 * checksum is verified too).  CHR_E_CORRUPT on any mismatch. */
int chr_stream_info(const void *h_stream, size_t n, chr_info *out);

/* Verifies every checksum of a whole stream held on the host. */
int chr_stream_verify(const void *h_stream, size_t n);

/* ---- reconstruction (Sec. II: the visualization side requests the data an
 *      isovalue needs at a desired accuracy) -------------------------------- */

/* Workspace bytes chr_reconstruct needs for this stream and level. */
size_t chr_reconstruct_workspace(const chr_info *info, int level);

/* Reconstructs level `level` of a stream held on the device (d_stream
 * 8-byte aligned, else CHR_E_INVAL).
 * info: header parsed by chr_stream_info from a host copy of the stream.
 * Output: d_out, float32 [((nz-1)>>level)+1][((ny-1)>>level)+1][((nx-1)>>level)+1],
 *   the reconstructed values of the points whose coordinates are multiples
 *   of 2^level.  Level 0 is the full field.
 * error_bound: the accuracy requested; must be >= the stream's bound
 *   (else CHR_E_ACCURACY).  level must be < levels (else CHR_E_LEVEL).
 * d_status: optional device int32, set to CHR_E_CORRUPT if a section fails
 *   its structural checks on the device (those sections are skipped). */
int chr_reconstruct(const chr_info *info, const void *d_stream, size_t stream_bytes,
                    int level, double error_bound, float *d_out, int32_t *d_status,
                    void *d_ws, size_t ws_bytes, void *stream);

/* Reconstruction restricted to what isosurfaces at isovalues in [kmin, kmax]
 * need (Sec. II.A: the block index lets the viewer touch only the blocks an
 * isovalue needs).  Blocks whose block-table range [min, max] admits no k in
 * [kmin, kmax] with min < k <= max are not decoded; their owned points get a
 * single value on the same side of every such k (the block's min or max).
 * For every isovalue k in [kmin, kmax], iso_extract / iso_cases on the result
 * give exactly what they give on the full chr_reconstruct output; the other
 * values are only guaranteed in reconstructed blocks.  Arguments, output and
 * errors as chr_reconstruct, plus CHR_E_INVAL for a non-finite or empty
 * range. */
int chr_reconstruct_range(const chr_info *info, const void *d_stream, size_t stream_bytes,
                          int level, double error_bound, float kmin, float kmax, float *d_out,
                          int32_t *d_status, void *d_ws, size_t ws_bytes, void *stream);

/* Bytes of the device array chr_reconstruct_static keeps the coarser-level
 * grids in (one copy per GPU, held until the process ends). */
#define CHR_STATIC_SCRATCH_BYTES ((size_t)96 << 20)

/* chr_reconstruct without a workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): the compact grids of the coarser levels
 * live in a library-owned device array of CHR_STATIC_SCRATCH_BYTES per GPU
 * (enough for level 0 of fields up to about 1.7e8 points, e.g. 512^3).
 * Arguments, output and errors as chr_reconstruct, plus CHR_E_NOMEM (nothing
 * launched) when the level needs more than the array holds.  Calls no
 * device allocation; the first call on a device looks the array's address up
 * (hipGetSymbolAddress), so make that first call outside a graph capture.
 * Every call on a GPU shares that GPU's array: calls that overlap on one GPU
 * (several streams or threads) race, so serialise them. */
int chr_reconstruct_static(const chr_info *info, const void *d_stream, size_t stream_bytes,
                           int level, double error_bound, float *d_out, int32_t *d_status,
                           void *stream);

/* ---- isosurface extraction (marching cubes, Sec. I and Sec. II.B) ------- */

/* Workspace bytes iso_extract / iso_cases need for a field of these dims. */
size_t iso_workspace(const int64_t dims[3]);

/* Marching cubes on d_field at `isovalue`.
 * Vertices: float32 [V][3] (x, y, z) in units of `spacing` grid steps
 *   (spacing 2^l for a level-l reconstruction), ordered by (grid point in
 *   x-fastest order, axis x<y<z) of the edge they lie on.
 * Triangles: int32 [T][3] vertex ids, ordered by cell, then table order;
 *   oriented with normals toward increasing field values.
 * d_counts: device int64[2] = {V, T}, the required sizes, written even when
 *   cap_v or cap_t is too small (then only the first cap_* are written).
 * Ids are int32: V beyond 2^31-1 is reported in d_counts and not written. */
int iso_extract(const float *d_field, const int64_t dims[3], float isovalue, float spacing,
                float *d_vertices, int64_t cap_v, int32_t *d_tris, int64_t cap_t,
                int64_t *d_counts, void *d_ws, size_t ws_bytes, void *stream);

/* Marching cubes' classification bits (Sec. II.B: the sign of value minus
 * isovalue at every vertex, which fixes every cell's case): one plane per
 * isovalue of dims[0] * dims[1] * ceil(dims[2] / 64) little-endian u64
 * words, row (z, y) at word (z * dims[1] + y) * ceil(dims[2] / 64), bit i of
 * word w = [value at x = 64 w + i < isovalue] (0 past the row's end). */

/* Level-0 reconstruction (as chr_reconstruct at level 0) that also writes
 * the classification bits of n_iso (1..16) isovalues into d_bits (n_iso
 * planes, plane j for h_isovalues[j], converted to binary32 as given).  The
 * level-0 decoder for 64-cell blocks writes them with the rows it decodes,
 * so marching cubes needs no pass over the field; otherwise one pass per
 * isovalue over the output follows.  Same workspace and errors as
 * chr_reconstruct, plus CHR_E_INVAL for a bad n_iso, non-finite isovalues or
 * a NULL d_bits. */
int chr_reconstruct_bits(const chr_info *info, const void *d_stream, size_t stream_bytes, double error_bound,
                         const float *h_isovalues, int n_iso, float *d_out, uint64_t *d_bits, int32_t *d_status,
                         void *d_ws, size_t ws_bytes, void *stream);

/* iso_extract of isovalue on d_field given its classification bits d_bits
 * (one plane as chr_reconstruct_bits writes, for this same isovalue):
 * identical outputs, without the pass over the field.  Same arguments,
 * workspace and errors as iso_extract. */
int iso_extract_bits(const float *d_field, const int64_t dims[3], const uint64_t *d_bits, float isovalue,
                     float spacing, float *d_vertices, int64_t cap_v, int32_t *d_tris, int64_t cap_t,
                     int64_t *d_counts, void *d_ws, size_t ws_bytes, void *stream);

/* Marching-cubes case of every cell: d_cases is uint8 [nz-1][ny-1][nx-1];
 * bit v is set iff the value at corner v = dx + 2dy + 4dz is below the
 * isovalue (f < k). */
int iso_cases(const float *d_field, const int64_t dims[3], float isovalue,
              uint8_t *d_cases, void *d_ws, size_t ws_bytes, void *stream);

/* Block merging for extraction (Sec. II.A: blocks merged into a larger
 * rectangular grid to be visualized more efficiently): the bounding box
 * lo..hi (z, y, x; inclusive level-0 points) of the blocks whose block-table
 * range [min, max] admits a crossing of some k in [kmin, kmax] (min < max,
 * min < kmax, kmin <= max).  h_head: host copy of the stream's header and
 * tables (payload_offset bytes).  *found = 0 (box untouched) when no block
 * qualifies.  Every cell with a crossing of such a k lies in the box, so
 * iso_extract_box over it gives iso_extract's mesh of the full field.
 * Errors: CHR_E_INVAL (NULL, empty or non-finite range), CHR_E_CORRUPT. */
int chr_block_box(const void *h_head, size_t head_bytes, float kmin, float kmax, int64_t lo[3], int64_t hi[3],
                  int *found);

/* Workspace bytes of iso_extract_box for a box of these dims (iso_workspace
 * of the box: the box is read in place). */
size_t iso_box_workspace(const int64_t box_dims[3]);

/* Marching cubes over the box lo..hi (z, y, x; inclusive, inside dims) of
 * d_field, with the field's coordinates: vertices and triangles as
 * iso_extract, ids in the box's point order (the field's order restricted to
 * the box).  When every cell with a crossing of `isovalue` lies in the box
 * (chr_block_box), the mesh equals iso_extract's on the whole field. */
int iso_extract_box(const float *d_field, const int64_t dims[3], const int64_t lo[3], const int64_t hi[3],
                    float isovalue, float spacing, float *d_vertices, int64_t cap_v, int32_t *d_tris, int64_t cap_t,
                    int64_t *d_counts, void *d_ws, size_t ws_bytes, void *stream);

/* Host copy of the library's generated triangle table:
 * ntri[256]; tri[256][15] cell-edge ids (unused entries -1). */
int chr_mc_table(uint8_t *ntri, int8_t *tri);

/* ---- error translation (Sec. II.B, the paper's three steps) -------------- */

/* Device scratch bytes chr_topology_error_bound needs (a few KB). */
size_t chr_topology_workspace(void);

/* The paper's translation of topology preservation into an error bound:
 * (1) find every grid edge (two points adjacent along x, y or z) whose end
 *     values s0 <= s1 enclose an isovalue k strictly, s0 < k < s1;
 * (2) collect d0 = k - s0 and d1 = s1 - k (in double) of each such edge and
 *     isovalue into the multiset D (isovalues as given, duplicates counted);
 * (3) return the nth smallest entry of D: nth <= 1 gives min(D), which keeps
 *     every crossing edge crossing; a larger nth tolerates the crossings of
 *     the smaller entries changing (a topology accuracy below 100%).
 * nth above |D| selects the largest entry.  d_out: device double[2] =
 * {bound, |D|}; the bound is +inf when D is empty.  Non-finite field values
 * never enclose an isovalue.  Asynchronous; d_ws holds the selection state
 * (chr_topology_workspace bytes). */
int chr_topology_error_bound(const float *d_field, const int64_t dims[3], const float *h_isovalues,
                             int n_iso, int64_t nth, double *d_out, void *d_ws, size_t ws_bytes,
                             void *stream);

/* ---- range (validation helper for relative error bounds) ---------------- */

/* Range of n values (Sec. II.B error translation works in absolute units; a
 * relative bound is rel * (max - min)).  d_out is 4 device words:
 * [0] min and [1] max of the finite values (float32), [2] number of
 * non-finite values (uint32), [3] unused. */
int chr_range(const float *d_field, int64_t n, float *d_out, void *stream);

/* ---- tile shapes ----------------------------------------------------------- */

/* Work distribution of the level-0 kernels: chunks (64 points) per wave for
 * compression (1, 2, 4, 8 or 16) and for reconstruction (8, 16, 32 or 64).
 * Results never depend on these; they apply to calls issued afterwards from
 * any thread of the process (not for use while another thread launches). */
int chr_set_tiles(int enc_chunks_per_wave, int dec_chunks_per_wave);

/* Which level-0 kernels run for 64-cell blocks: 1 (default) = one workgroup
 * per pair of z-planes of a block, rows along x, codes gathered in LDS and
 * packed per chunk; 0 = one wave per 64-point chunk (the kernels every other
 * block size uses).  Results never depend on it; same scope as
 * chr_set_tiles.  CHR_E_INVAL for any other value. */
int chr_set_level0_tiles(int on);

/* ---- batches (many fields of uneven sizes in one captured launch) --------- */

/* The per-field workflow of Sec. II (compress with the topology check of
 * Sec. II.B, reconstruct, extract the isosurfaces) applied to many fields at
 * once: timesteps or bricks of uneven sizes, each with its own isovalues.
 * Nothing in the arithmetic changes: every item runs the same kernels with
 * the same launch plans as chr_compress (no codes/flags output),
 * chr_reconstruct_bits for its isovalues and iso_extract_bits, so each of its
 * outputs is bit for bit what chr_compress, chr_reconstruct at level 0 and
 * iso_extract give.  Its field is not read again for classification: the
 * level-0 decoder writes every isovalue's bits as it reconstructs. */

/* One field of a batch.  All pointers are caller-owned device buffers that
 * must stay valid while the batch (or its captured graph) is in use. */
typedef struct chr_batch_item {
  const float *d_field;        /* float32 [dims[0]][dims[1]][dims[2]], x fastest */
  int64_t dims[3];
  double error_bound;          /* absolute, >= 0 (0 = lossless) */
  int n_iso;                   /* 0..16 */
  float isovalues[16];         /* candidates protected by compression, each extracted in order */
  chr_params params;
  void *d_stream;              /* stream output, stream_capacity bytes (chr_compress_bound suffices) */
  size_t stream_capacity;
  chr_result *d_result;        /* as chr_compress's */
  float *d_recon;              /* level-0 reconstruction, same dims as the field */
  float *d_vertices[16];       /* mesh of isovalue j: vertices [cap_v[j]][3], triangles ... */
  int64_t cap_v[16];
  int32_t *d_tris[16];         /* ... [cap_t[j]][3] (either may be NULL with capacity 0) ... */
  int64_t cap_t[16];
  int64_t *d_counts;           /* ... and {V, T} of isovalue j at d_counts[2j] (int64 [n_iso][2]) */
  int32_t *d_status;           /* optional: reconstruction status, reset to 0 by every run */
  float spacing;               /* grid spacing of the extracted vertices */
} chr_batch_item;

typedef struct chr_batch chr_batch;

/* Plans a batch (host only, no device call; items are copied).  Items are
 * spread over min(8, n_items) parallel branches by default (see
 * chr_batch_set_config), longest first onto the least-loaded branch;
 * level-0 tiles are those of chr_set_tiles at creation.  Errors: CHR_E_INVAL (bad parameters, NULL
 * pointer, bad mesh capacity; chr_last_error names the item),
 * CHR_E_CAPACITY (stream capacity below the header and tables). */
int chr_batch_create(const chr_batch_item *items, int n_items, chr_batch **out);

/* Device scratch bytes the batch needs for any branch count and tile shape
 * (one region per branch; items of a branch reuse it in turn). */
size_t chr_batch_workspace(const chr_batch *b);

/* Launches the whole batch on `stream`: forked over the branches' own
 * streams with an event and joined back into `stream` with one.  Stream
 * overflow and non-finite input are reported per item in d_result, as by
 * chr_compress; a corrupt section in d_status. */
int chr_batch_run(chr_batch *b, void *d_ws, size_t ws_bytes, void *stream);

/* Captures the same launches into a HIP graph (replacing any earlier one;
 * `stream` is unused: capture happens on a stream of the batch's own).  The
 * graph keeps the workspace address; nothing runs until a replay. */
int chr_batch_capture(chr_batch *b, void *d_ws, size_t ws_bytes, void *stream);

/* Launches the captured graph on `stream` (CHR_E_INVAL before a capture). */
int chr_batch_replay(chr_batch *b, void *stream);

/* Switched off (returns CHR_E_INVAL; chr_batch_tune replaces it): one GPU
 * run aborted inside its replay-timed search and the cause is not known.
 * Chose the branch count (1, 2, 4, 8) and the level-0 tiles
 * (chr_set_tiles' candidates) by timing replays of the captured batch:
 * coordinate descent from the current configuration over branches, then
 * compression tiles, then reconstruction tiles; a change is kept when it is
 * at least 1% faster.  Ends with the chosen configuration captured.
 * cache_path (may be NULL): text file of "signature branches enc dec" lines,
 * signature = hash of the items' shapes and parameters and the device; a
 * matching line skips the search, a new result is appended. */
int chr_batch_autotune(chr_batch *b, void *d_ws, size_t ws_bytes, void *stream, const char *cache_path);

/* Chooses the brick size B of every item's stream (as created, 32, 64 or
 * 128: Sec. II.A's blocks; B changes the stream bytes, never a reconstructed
 * value or a mesh), the branch count (1, 2, 4, 8) and the level-0 tiles by
 * timing eager runs of the whole batch on `stream` (two per candidate, after
 * an untimed one): coordinate descent over B, branches, compression tiles,
 * reconstruction tiles from the current configuration; a change is kept when
 * at least 1% faster.  A block size invalid for an item (not a multiple of
 * 2^(levels-1)), a stream bound above an item's stream_capacity or a
 * workspace above ws_bytes skips that candidate.  Ends with the chosen
 * configuration captured (as chr_batch_capture).  *block_out (may be NULL):
 * the chosen B, 0 for each item's own.  cache_path (may be NULL): text file
 * of "signature branches block enc dec" lines; a matching line skips the
 * search, a new result is appended.  The outputs hold the last timed run's
 * results.  Errors: CHR_E_INVAL, CHR_E_NOMEM (workspace too small for the
 * configuration as created), CHR_E_HIP. */
int chr_batch_tune(chr_batch *b, void *d_ws, size_t ws_bytes, void *stream, const char *cache_path,
                   int *block_out);

/* Current configuration and the duration of the last timed replay (ms). */
int chr_batch_config(const chr_batch *b, int *branches, int *enc_cpw, int *dec_cpw, float *last_ms);

/* Sets the configuration by hand (branches 1 .. min(8, n_items); tiles as in
 * chr_set_tiles) for the next chr_batch_run or chr_batch_capture; an earlier
 * capture keeps its own until captured again.  Host only.  Errors:
 * CHR_E_INVAL (NULL batch, a value out of range; nothing changes). */
int chr_batch_set_config(chr_batch *b, int branches, int enc_cpw, int dec_cpw);

/* Releases the batch's streams, events and graph (not the caller's buffers). */
int chr_batch_destroy(chr_batch *b);

/* ---- serving (resident streams, continuous batching) ---------------------- */

/* The visualization side of Sec. II: a viewer asks for the isosurface of a
 * dataset at an isovalue and an accuracy, and the data it needs is
 * reconstructed from the CHR held in memory (here: resident in HBM) and
 * isosurfaced.  A request (dataset, isovalue, accuracy, level) is served
 * from the dataset's stream with the largest error bound <= accuracy,
 * reconstructed at `level` and extracted with spacing 2^level.
 *
 * Continuous batching: queued requests are admitted whenever a slot (a HIP
 * stream of the server's own) and pool memory are free.  Requests with the
 * same (stream, level) at the head of the queue form a group sharing one
 * reconstruction; each request of a group then runs the counting half of
 * marching cubes, the host reads the counts, allocates exactly sized lists
 * and mesh from the pool, and launches the emitting half.  Groups on
 * different slots overlap on the device.  Admission is FIFO by memory
 * footprint: reconstruction + its workspace + per-request counting state
 * must fit in the pool, else the head of the queue waits until completed
 * work frees memory.  Every request runs the kernels and arithmetic of
 * chr_reconstruct + iso_extract, so its mesh is bit for bit what those calls
 * give, alone or in any mix.
 *
 * All calls are host calls on one thread (the server is not thread-safe).
 * create/add_stream/submit/poll/cancel/release make no HIP call; step and
 * destroy do. */

typedef struct chr_server chr_server;

typedef struct chr_server_config {
  int slots;            /* groups in flight at once, 1..16 */
  int max_group;        /* requests sharing one reconstruction, 1..64 */
  void *d_pool;         /* caller-owned device memory the server allocates from */
  size_t pool_bytes;
} chr_server_config;

typedef struct chr_request_result {
  int32_t status;       /* CHR_PENDING, CHR_OK, CHR_E_CANCELLED, CHR_E_NOMEM, CHR_E_CORRUPT, CHR_E_HIP */
  int32_t level;
  int32_t dataset;
  int32_t stream_index; /* which registered stream served it */
  float isovalue;
  int32_t group_size;   /* requests that shared its reconstruction */
  double error_bound;   /* of that stream */
  int64_t n_vertices, n_triangles;
  const float *d_vertices;     /* float32 [n_vertices][3] in the pool, valid until release */
  const int32_t *d_triangles;  /* int32 [n_triangles][3] in the pool, valid until release */
  double t_submit_ms, t_admit_ms, t_done_ms;  /* server clock (chr_server_now_ms) */
} chr_request_result;

typedef struct chr_server_stats {
  int64_t queued, in_flight, done, failed;
  size_t pool_used, pool_peak;
  int64_t groups, grouped_requests;
} chr_server_stats;

/* Errors: CHR_E_INVAL (slots or max_group out of range, NULL pool). */
int chr_server_create(const chr_server_config *cfg, chr_server **out);

/* Registers a resident stream of `dataset` (any int id).  info: parsed by
 * chr_stream_info from a host copy of the stream's header and tables;
 * d_stream (caller-owned, stream_bytes >= info->total_bytes) must stay valid
 * and unchanged while the server lives.  *index: the stream's index. */
int chr_server_add_stream(chr_server *s, int dataset, const chr_info *info, const void *d_stream,
                          size_t stream_bytes, int *index);

/* Queues a request; *id identifies it.  Errors (nothing queued):
 * CHR_E_INVAL unknown dataset or non-finite isovalue; CHR_E_ACCURACY no
 * stream of the dataset meets `accuracy`; CHR_E_LEVEL level outside that
 * stream's hierarchy; CHR_E_NOMEM its footprint exceeds the whole pool. */
int chr_server_submit(chr_server *s, int dataset, float isovalue, double accuracy, int level, int64_t *id);

/* Advances every group whose device work has finished and admits queued
 * requests into free slots; never waits for the device.  *n_done (may be
 * NULL): requests that finished in this call. */
int chr_server_step(chr_server *s, int *n_done);

/* State of a request (CHR_E_INVAL for an unknown or released id). */
int chr_server_poll(const chr_server *s, int64_t id, chr_request_result *out);

/* Frees a finished request's mesh; its id becomes unknown. */
int chr_server_release(chr_server *s, int64_t id);

/* Cancels a request: a queued one leaves the queue, one in flight has its
 * outputs freed when its group finishes.  Its status becomes CHR_E_CANCELLED. */
int chr_server_cancel(chr_server *s, int64_t id);

int chr_server_stats_get(const chr_server *s, chr_server_stats *out);
double chr_server_now_ms(const chr_server *s);

/* Waits for work in flight, then frees the server's streams, events and
 * pinned host memory (not the pool). */
int chr_server_destroy(chr_server *s);

/* ---- measurement support ------------------------------------------------ */

/* While enabled, every launch of the kernel named `kernel` (for example
 * "k_encode_fine") records a HIP event before and after it on its launch
 * stream, up to max_launches launches.  chr_prof_collect returns the
 * durations in milliseconds of the launches recorded so far (the caller must
 * have synchronized the stream) and starts a new collection; chr_prof_disable
 * releases the events.  Host-side; not thread-safe. */
int chr_prof_enable(const char *kernel, int max_launches);
int chr_prof_collect(float *ms, int max, int *n_out);
int chr_prof_disable(void);

/* ---- entropy stage (the stream on the network leg, Sec. III) -------------
 *
 * An order-0 canonical Huffman code over the bytes of any byte string (a CHR
 * stream in practice), in independently decodable 512-byte chunks.  Code
 * lengths: Huffman's two-queue construction over the byte counts (ties: the
 * smaller count, then the smaller byte value, a leaf before an internal node
 * of equal weight), limited to 12 bits by the JPEG rule (ITU-T T.81 Annex
 * K.3), then given to the byte values from the most frequent; codes:
 * RFC 1951 Sec. 3.2.2 canonical assignment.  Layout (little-endian):
 *   0 u32 "CHRH"  4 u32 version 1  8 u64 n  16 u32 chunk bytes (512)
 *   20 u32 nchunks = ceil(n / 512)  24 u64 total bytes  32 u32 max length 12
 *   36..63 zero; 64 u8 code length of each byte value (0: absent)
 *   320 u32 word offset of each chunk's bits (nchunks + 1 entries, the last
 *   being the bit area's length in words), zero padding to 8 bytes
 *   bit area: each chunk's codes from its word offset, bits LSB-first within
 *   32-bit words, each code most-significant bit first; last word zero-padded.
 * Inputs and outputs are device buffers, 8-byte aligned; n < 2^32. */

/* Encoded size bound of n bytes (the capacity that always suffices). */
size_t chr_entropy_bound(uint64_t n);
/* Device workspace of chr_entropy_encode for n bytes. */
size_t chr_entropy_workspace(uint64_t n);
/* Encodes d_in[0 .. n).  d_result: 2 device words, [0] the encoded size
 * (the required size when [1] = CHR_E_CAPACITY), [1] 0 or CHR_E_CAPACITY
 * (nothing but the result is written then).  Errors: CHR_E_INVAL (NULL or
 * misaligned pointer, n >= 2^32), CHR_E_NOMEM (workspace too small). */
int chr_entropy_encode(const void *d_in, uint64_t n, void *d_out, size_t capacity, uint64_t *d_result, void *d_ws,
                       size_t ws_bytes, void *stream);
/* Parses the first 64 bytes of an encoded stream (host copy): decoded size n
 * and encoded size.  CHR_E_CORRUPT if they are not a version-1 header with
 * 512-byte chunks and 12-bit codes. */
int chr_entropy_info(const void *h_head, size_t head_bytes, uint64_t *n, uint64_t *total);
/* Decodes the encoded stream d_in (nbytes, its header also on the host as
 * h_head) into d_out[0 .. n).  Codes are read canonically (the shortest
 * length whose prefix is a code of that length), so any length table
 * decodes deterministically.  *d_status is set to 0, or CHR_E_CORRUPT when a
 * chunk's offsets or codes are invalid or a stored length exceeds 12.
 * Errors: as chr_entropy_info,
 * CHR_E_CAPACITY (out_capacity < n), CHR_E_INVAL (NULL or misaligned). */
int chr_entropy_decode(const void *h_head, const void *d_in, uint64_t nbytes, void *d_out, uint64_t out_capacity,
                       int32_t *d_status, void *stream);

/* ---- Multi-tier progressive accuracy (Sec. II: data at the accuracy the
 * viewer requests) ----------------------------------------------------------
 * Tier 0 is the topology-preserving stream of the field at bound[0]; tier t
 * >= 1 is the stream, without isovalues, of the binary32 residual
 * x - y_{t-1} at bound[t] (y_{t-1}: the reconstruction from tiers 0..t-1),
 * plus, in index order, the index and value of every point where
 * y_{t-1} + r'_t (binary32) misses bound[t] (checked in double) or lies on
 * another side of a candidate isovalue than x; those points take x.  A
 * reconstruction at an accuracy eb decodes tiers 0..t for the first t with
 * bound[t] <= eb.
 * Container (little-endian): 0 u32 "CHRT", 4 u32 version 1, 8 u32 tiers,
 * 12 u32 candidate count, 16 i64 dims[3], 40 u32 levels, 44 u32 block,
 * 48 u32 qmax, 56 f32 isovalues[16], 120 u64 total bytes; at 128, 8 records
 * of 64 bytes (f64 bound, u64 stream offset, stream bytes, corrections,
 * index offset, value offset, 16 zero); from 640 each tier's stream, u64
 * indices and f32 values, every part 8-aligned and zero-padded. */
#define CHR_MAX_TIERS 8

typedef struct chr_tier_header {
  int n_tiers, n_iso;
  int64_t dims[3];
  int levels, block, qmax, reserved;
  float isovalues[16];
  uint64_t total_bytes;
  double bound[CHR_MAX_TIERS];
  uint64_t stream_offset[CHR_MAX_TIERS], stream_bytes[CHR_MAX_TIERS], n_corrections[CHR_MAX_TIERS];
  uint64_t index_offset[CHR_MAX_TIERS], value_offset[CHR_MAX_TIERS];
} chr_tier_header;

/* Largest container of n_tiers tiers (0 and chr_last_error on bad parameters). */
size_t chr_tiers_bound(const int64_t dims[3], int n_tiers, const chr_params *params);
/* Device scratch bytes of chr_tiers_compress: two fields, one tier stream and
 * the single-field compression and reconstruction workspaces. */
size_t chr_tiers_workspace(const int64_t dims[3], const chr_params *params);
/* Builds the container of `d_field` (float32, dims as chr_compress) on
 * `stream`.  bounds: 1..CHR_MAX_TIERS host values, finite, >= 0, strictly
 * decreasing; params.error_bound_far must be 0.  d_out (8-byte aligned,
 * `capacity` bytes) receives the container; d_result (2 x uint64, device,
 * 8-byte aligned) the container size (the required size when it does not
 * fit) and the status (0, CHR_E_INVAL for non-finite input, CHR_E_CAPACITY).
 * Host errors: CHR_E_INVAL, CHR_E_NOMEM (workspace), CHR_E_CAPACITY (below
 * the 640-byte header). */
int chr_tiers_compress(const float *d_field, const int64_t dims[3], const double *h_bounds, int n_tiers,
                       const float *h_isovalues, int n_iso, const chr_params *params, void *d_out, size_t capacity,
                       uint64_t *d_result, void *d_ws, size_t ws_bytes, void *stream);
/* Parses the first 640 bytes of a container (host copy); CHR_E_CORRUPT when
 * they are not a consistent tier header. */
int chr_tiers_header(const void *h_head, size_t head_bytes, chr_tier_header *out);
/* Device scratch bytes of chr_tiers_reconstruct. */
size_t chr_tiers_reconstruct_workspace(const chr_tier_header *header);
/* Reconstructs the full-resolution field at accuracy error_bound from the
 * fewest tiers that meet it (CHR_E_ACCURACY when none does); *tier_used
 * (host, may be NULL) receives the last tier decoded.  d_container is the
 * whole container on the device (8-byte aligned, `bytes` long); d_status (one
 * int32 on the device) is set to 0, or CHR_E_CORRUPT when a stream or a
 * correction index is inconsistent. */
int chr_tiers_reconstruct(const chr_tier_header *header, const void *d_container, size_t bytes, double error_bound,
                          float *d_out, int32_t *d_status, void *d_ws, size_t ws_bytes, int *tier_used, void *stream);

#ifdef __cplusplus
}
#endif
#endif
