/*
 * chr_oracle.h -- CPU oracle for the Compressed Hierarchical Representation (CHR)
 * and marching cubes.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never links, loads or calls it.  It shares no code with the
 * GPU library (no headers, tables, helpers or generators).
 *
 * Paper: "Accelerating In-transit Isosurface Generation With Topology
 * Preserving Compression" (arXiv 2408.05462).  The paper fixes
 *   - topology preservation: the decompressed field must give every cell the
 *     same marching-cubes case (Sec. II.B, definition of topology
 *     preservation);
 *   - the sufficient condition: an error smaller than both vertex-to-isovalue
 *     distances d0, d1 keeps the case (Sec. II.B, edge condition);
 *   - the error translation over the array D of those distances and its
 *     relaxation to the n-th smallest entry (Sec. II.B, three-step procedure).
 * Everything else (hierarchy, predictor, quantizer, stream format, triangle
 * table) is unspecified in the paper; the readings implemented here are listed
 * in the design notes and in each function's comment.
 *
 * Conventions: a field is float32 [nz][ny][nx], x fastest; dims[] = {nz,ny,nx}.
 * Parity unpinned: compression ratio (the paper prints none).
 */
#ifndef CHR_ORACLE_H
#define CHR_ORACLE_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORC_OK = 0,
  ORC_E_INVAL = -1,
  ORC_E_ACCURACY = -2,
  ORC_E_LEVEL = -3,
  ORC_E_CORRUPT = -4,
  ORC_E_CAPACITY = -5,
  ORC_E_NOMEM = -6
};

/* Number of threads the oracle's parallel loops use. */
int orc_threads(void);

/* Level of grid point (x,y,z) in an nL-level hierarchy (reading R4). */
int orc_level_of(int64_t x, int64_t y, int64_t z, int nL);

/* Multilinear midpoint prediction of point (x,y,z) at level l from the
 * reconstructed values in xr (a full [nz][ny][nx] array), reading R6. */
float orc_predict(const float *xr, const int64_t dims[3], int64_t x, int64_t y,
                  int64_t z, int level, int nL);

/* Error-bounded linear quantization of one value (reading R7).  Writes the
 * code q, the outlier flag and the reconstructed value. */
void orc_quantize(float x, float p, double e, int qmax, int32_t *q, int *outlier,
                  float *xr);

/* Number of (sorted) candidate isovalues k with k <= v (reading R2). */
int orc_rank(float v, const float *iso, int n_iso);

/* Maximum stream size for a field of these dims and parameters. */
size_t orc_compress_bound(const int64_t dims[3], int nL, int block);

/* Full compression.  q_out/flags_out/xr_out are per-point arrays in field
 * layout (may be NULL): q is the quantization code (0 where the value is
 * stored exactly), flags bit0 = outlier (O), bit1 = topology correction (C),
 * xr = reconstructed value.  Writes the stream into `stream` (capacity cap),
 * its size into *stream_bytes (the required size on ORC_E_CAPACITY).
 * error_bound_far = 0: one bound everywhere; otherwise (finite, >= error_bound)
 * differentiated error control (reading R19): points of no block crossing a
 * candidate isovalue are quantized with the far bound. */
int orc_compress(const float *x, const int64_t dims[3], double error_bound, double error_bound_far,
                 const float *iso, int n_iso, int nL, int block, int qmax,
                 int32_t *q_out, uint8_t *flags_out, float *xr_out,
                 uint8_t *stream, size_t cap, size_t *stream_bytes);

/* Compression with block merging before compression (Sec. II.A, third
 * step; reading R22): merge = the largest number of blocks per axis of a
 * merged unit (0 or 1: no merging, the stream of orc_compress).  Blocks
 * with equal index signatures (the set of candidate isovalues their input
 * range crosses) are merged greedily into rectangular units, each stored as
 * one closed extent; codes and reconstruction are those of orc_compress.
 * Not combined with error_bound_far (ORC_E_INVAL). */
int orc_compress_merged(const float *x, const int64_t dims[3], double error_bound, double error_bound_far,
                        const float *iso, int n_iso, int nL, int block, int qmax, int merge,
                        int32_t *q_out, uint8_t *flags_out, float *xr_out,
                        uint8_t *stream, size_t cap, size_t *stream_bytes);

/* Stream size bound with merging (adds the box table). */
size_t orc_compress_bound_merged(const int64_t dims[3], int nL, int block, int merge);

/* Header fields of a stream (after checksum validation).  nblocks counts the
 * storage units (blocks, or merged units when flags bit 3 is set). */
typedef struct {
  int64_t dims[3];
  int levels, block, qmax, n_iso;
  double error_bound;
  float inv, step;
  float iso[16];
  float vmin, vmax;
  int64_t nblocks;
  int nb[3];
  uint32_t flags;
  uint64_t total_bytes, n_outlier, n_corrected, payload_offset;
  double error_bound_far;  /* flags bit 1: differentiated error control */
  float inv_far, step_far;
  int merge;               /* flags bit 3: largest blocks per axis of a unit (1: no merging) */
  int mb[3];               /* largest unit extent in blocks along z, y, x */
} orc_info;

int orc_stream_info(const uint8_t *stream, size_t n, orc_info *out);

/* Verify every checksum of a whole stream; ORC_OK or ORC_E_CORRUPT. */
int orc_stream_verify(const uint8_t *stream, size_t n);

/* Per-point codes and exact-storage mask of a stream, read back from its
 * sections (codes of points stored exactly are 0).  Output arrays are in field
 * layout; every point gets the value from the block that owns it. */
int orc_stream_codes(const uint8_t *stream, size_t n, int32_t *q_out,
                     uint8_t *e_out);

/* Reconstruction to `level` (reading R10): output dims ((n-1)>>level)+1.
 * Each closed block is decoded on its own from its sections only. */
int orc_decompress(const uint8_t *stream, size_t n, int level, double error_bound,
                   float *out);

/* Per-block min/max of the reconstructed values as stored in the block table. */
int orc_block_index(const uint8_t *stream, size_t n, float *mins, float *maxs);

/* Marching-cubes table generated from the face rule (reading R12).
 * ntri[c] triangles for case c; tri[c][3*t+i] = cell edge id (0..11). */
#define ORC_MC_MAXTRI 12
void orc_mc_table(uint8_t ntri[256], int8_t tri[256][3 * ORC_MC_MAXTRI]);

/* Case index of every cell (reading R1): bit v set iff f(corner v) < k,
 * corner v = dx + 2dy + 4dz.  cases is [nz-1][ny-1][nx-1]. */
void orc_mc_cases(const float *f, const int64_t dims[3], float k, uint8_t *cases);

/* Marching cubes (Sec. I, II.B).  Vertices ordered by (point, axis),
 * triangles by (cell, table order), reading R13.  Positions in units of
 * `spacing` (reading R11).  counts[0]=vertices, counts[1]=triangles (the
 * required sizes even when the capacities are too small). */
int orc_mc(const float *f, const int64_t dims[3], float k, float spacing,
           float *verts, int64_t cap_v, int32_t *tris, int64_t cap_t,
           int64_t counts[2]);

/* Paper's error translation (Sec. II.B, three steps): collect d0 = k - s0 and
 * d1 = s1 - k over every edge with s0 < k < s1 (either orientation) into D and
 * return the n-th smallest (1-based n; n = 1 gives min(D)).  Returns the size
 * of D in *n_d; the result is +inf when D is empty. */
double orc_topology_error_bound(const float *f, const int64_t dims[3],
                                const float *iso, int n_iso, int64_t nth,
                                int64_t *n_d);

/* Block merging for extraction: bounding box (z, y, x; inclusive) of the
 * blocks whose stored range can hold a crossing of an isovalue in
 * [kmin, kmax]; *found = 0 when none can. */
int orc_block_box(const uint8_t *stream, size_t n, float kmin, float kmax, int64_t lo[3], int64_t hi[3], int *found);
/* Marching cubes over the box lo..hi of a field, positions in the field's coordinates. */
int orc_mc_box(const float *f, const int64_t dims[3], const int64_t lo[3], const int64_t hi[3], float k,
               float spacing, float *verts, int64_t cap_v, int32_t *tris, int64_t cap_t, int64_t counts[2]);

/* ---- entropy stage (chr_entropy.c): order-0 Huffman over a byte stream ---- */

/* Code lengths of the 256 byte values from their counts, at most maxlen
 * bits (8..31); 0 for absent values, 1 for a value that is alone. */
int orc_huff_lengths(const uint64_t hist[256], int maxlen, uint8_t len[256]);
/* Canonical codes of the lengths (most significant bit first). */
int orc_huff_codes(const uint8_t len[256], uint32_t code[256]);
/* Encoded size bound of n bytes. */
uint64_t orc_entropy_bound(uint64_t n, uint32_t chunk, int maxlen);
/* Encodes n bytes (chunk bytes per independently decodable chunk, a multiple
 * of 4; maxlen 8..24); *out_bytes receives the size (the required size on
 * ORC_E_CAPACITY). */
int orc_entropy_encode(const uint8_t *in, uint64_t n, uint32_t chunk, int maxlen, uint8_t *out, uint64_t cap,
                       uint64_t *out_bytes);
/* Decoded size and chunk bytes of an encoded stream (ORC_E_CORRUPT if it is not one). */
int orc_entropy_info(const uint8_t *in, uint64_t nbytes, uint64_t *n, uint32_t *chunk);
/* Decodes a whole encoded stream; *n_out receives the decoded size. */
int orc_entropy_decode(const uint8_t *in, uint64_t nbytes, uint8_t *out, uint64_t out_cap, uint64_t *n_out);

/* ---- multi-tier progressive accuracy (chr_tiers.c) ---- */

#define ORC_MAX_TIERS 8
/* Container size bound for T tiers. */
uint64_t orc_tiers_bound(const int64_t dims[3], int T, int nL, int block);
/* Tiers at bounds[0] > bounds[1] > ... >= 0 (T <= 8); *out_bytes receives the
 * container size (the required size on ORC_E_CAPACITY). */
int orc_tiers_compress(const float *x, const int64_t dims[3], const double *bounds, int T, const float *iso,
                       int n_iso, int nL, int block, int qmax, uint8_t *out, uint64_t cap, uint64_t *out_bytes);
/* Tier count, bounds and total size of a container. */
int orc_tiers_info(const uint8_t *in, uint64_t n, int *T, double *bounds, uint64_t *total);
/* Reconstruction at accuracy eb from the fewest tiers that meet it
 * (ORC_E_ACCURACY when no tier does); *tier_used receives the last tier. */
int orc_tiers_decompress(const uint8_t *in, uint64_t n, double eb, float *out, int *tier_used);

#ifdef __cplusplus
}
#endif
#endif
