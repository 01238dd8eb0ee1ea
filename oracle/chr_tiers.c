/*
 * chr_tiers.c -- CPU oracle of multi-tier progressive accuracy.
 *
 * TEST INFRASTRUCTURE ONLY, like chr_oracle.c: the reference the GPU tier
 * container is checked against.  It shares no code with the GPU library and
 * builds on this oracle's own compression and reconstruction.
 *
 * The paper lets the visualization side request data at a desired accuracy
 * (Sec. II, framework) without fixing how accuracies are layered.  Reading
 * used here (residual tiers):
 *   - bounds e_0 > e_1 > ... > e_{T-1} >= 0, at most 8 tiers;
 *   - tier 0 is the topology-preserving CHR stream of x at e_0 with the
 *     candidate isovalues; its reconstruction is y_0;
 *   - tier t >= 1 is the CHR stream at e_t, without isovalues, of the
 *     binary32 residual r_t = x - y_{t-1}; decoding it gives r'_t and the
 *     candidate y_t = y_{t-1} + r'_t (binary32);
 *   - every point where y_t misses e_t (checked in double) or lies on another
 *     side of a candidate isovalue than x is corrected: y_t = x there, and
 *     the tier stores the point's index and x, in index order;
 *   - reconstruction at an accuracy eb decodes tiers 0..t for the first t
 *     with e_t <= eb (CHR_E_ACCURACY-like error when there is none).
 *
 * Container (little-endian):
 *   0 u32 magic "CHRT"   4 u32 version 1   8 u32 T   12 u32 K
 *   16 i64 dims[3]   40 u32 levels   44 u32 block   48 u32 qmax   52 u32 0
 *   56 f32 isovalues[16] (sorted, distinct; tier 0's)   120 u64 total bytes
 *   128 tier records, 8 x 64 bytes: f64 e_t, u64 stream offset, u64 stream
 *       bytes, u64 corrections, u64 index offset, u64 value offset, 16 zero
 *   640 tier 0's stream, then its index list (u64) and value list (f32,
 *       padded to 8), then tier 1's, ...; every part starts 8-aligned.
 */
#include "chr_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define T_MAGIC 0x54524843u /* "CHRT" */
#define T_VERSION 1u
#define T_HEAD 128
#define T_REC 64
#define T_DATA (T_HEAD + T_REC * ORC_MAX_TIERS)

static void t_put32(uint8_t *p, uint32_t v) { for (int i = 0; i < 4; i++) p[i] = (uint8_t)(v >> (8 * i)); }
static void t_put64(uint8_t *p, uint64_t v) { for (int i = 0; i < 8; i++) p[i] = (uint8_t)(v >> (8 * i)); }
static uint32_t t_get32(const uint8_t *p) { uint32_t v = 0; for (int i = 0; i < 4; i++) v |= (uint32_t)p[i] << (8 * i); return v; }
static uint64_t t_get64(const uint8_t *p) { uint64_t v = 0; for (int i = 0; i < 8; i++) v |= (uint64_t)p[i] << (8 * i); return v; }
static void t_putd(uint8_t *p, double d) { uint64_t u; memcpy(&u, &d, 8); t_put64(p, u); }
static double t_getd(const uint8_t *p) { uint64_t u = t_get64(p); double d; memcpy(&d, &u, 8); return d; }
static uint64_t t_pad8(uint64_t n) { return (n + 7) & ~(uint64_t)7; }

uint64_t orc_tiers_bound(const int64_t dims[3], int T, int nL, int block) {
  const uint64_t N = (uint64_t)dims[0] * (uint64_t)dims[1] * (uint64_t)dims[2];
  const uint64_t per = t_pad8(orc_compress_bound(dims, nL, block)) + 8 * N + t_pad8(4 * N);
  return T_DATA + (uint64_t)T * per;
}

int orc_tiers_compress(const float *x, const int64_t dims[3], const double *bounds, int T, const float *iso_in,
                       int n_iso, int nL, int block, int qmax, uint8_t *out, uint64_t cap, uint64_t *out_bytes) {
  if (T < 1 || T > ORC_MAX_TIERS || !bounds) return ORC_E_INVAL;
  for (int t = 0; t < T; t++) {
    if (!(bounds[t] >= 0) || !isfinite(bounds[t])) return ORC_E_INVAL;
    if (t > 0 && !(bounds[t] < bounds[t - 1])) return ORC_E_INVAL;
  }
  const uint64_t N = (uint64_t)dims[0] * (uint64_t)dims[1] * (uint64_t)dims[2];
  const size_t sb = orc_compress_bound(dims, nL, block);
  if (sb == 0) return ORC_E_INVAL;
  float *y = (float *)malloc(sizeof(float) * N), *r = (float *)malloc(sizeof(float) * N);
  float *rr = (float *)malloc(sizeof(float) * N);
  uint8_t *s = (uint8_t *)malloc(sb);
  uint64_t *cidx = (uint64_t *)malloc(sizeof(uint64_t) * N);
  float *cval = (float *)malloc(sizeof(float) * N);
  uint8_t *buf = (uint8_t *)calloc(1, (size_t)orc_tiers_bound(dims, T, nL, block));
  int rc = ORC_OK;
  if (!y || !r || !rr || !s || !cidx || !cval || !buf) rc = ORC_E_NOMEM;
  orc_info I0;
  uint64_t off = T_DATA;
  for (int t = 0; t < T && rc == ORC_OK; t++) {
    size_t nb = 0;
    uint64_t nc = 0;
    if (t == 0) {
      /* tier 0: the topology-preserving stream of x */
      rc = orc_compress(x, dims, bounds[0], 0.0, iso_in, n_iso, nL, block, qmax, NULL, NULL, y, s, sb, &nb);
      if (rc) break;
      rc = orc_stream_info(s, nb, &I0);
      if (rc) break;
    } else {
      /* tier t: the residual against the previous tiers' reconstruction */
      for (uint64_t i = 0; i < N; i++) r[i] = x[i] - y[i];
      rc = orc_compress(r, dims, bounds[t], 0.0, NULL, 0, nL, block, qmax, NULL, NULL, NULL, s, sb, &nb);
      if (rc) break;
      rc = orc_decompress(s, nb, 0, bounds[t], rr);
      if (rc) break;
      for (uint64_t i = 0; i < N; i++) {
        const float v = y[i] + rr[i];
        const int bad = !(fabs((double)v - (double)x[i]) <= bounds[t]) ||
                        orc_rank(v, I0.iso, I0.n_iso) != orc_rank(x[i], I0.iso, I0.n_iso);
        if (bad) {
          cidx[nc] = i;
          cval[nc] = x[i];
          nc++;
          y[i] = x[i];
        } else {
          y[i] = v;
        }
      }
    }
    uint8_t *rec = buf + T_HEAD + T_REC * t;
    t_putd(rec, bounds[t]);
    t_put64(rec + 8, off);
    t_put64(rec + 16, nb);
    memcpy(buf + off, s, nb);
    off = t_pad8(off + nb);
    t_put64(rec + 24, nc);
    t_put64(rec + 32, off);
    for (uint64_t j = 0; j < nc; j++) t_put64(buf + off + 8 * j, cidx[j]);
    off = t_pad8(off + 8 * nc);
    t_put64(rec + 40, off);
    for (uint64_t j = 0; j < nc; j++) {
      uint32_t u;
      memcpy(&u, &cval[j], 4);
      t_put32(buf + off + 4 * j, u);
    }
    off = t_pad8(off + 4 * nc);
  }
  if (rc == ORC_OK) {
    t_put32(buf, T_MAGIC);
    t_put32(buf + 4, T_VERSION);
    t_put32(buf + 8, (uint32_t)T);
    t_put32(buf + 12, (uint32_t)I0.n_iso);
    for (int a = 0; a < 3; a++) t_put64(buf + 16 + 8 * a, (uint64_t)dims[a]);
    t_put32(buf + 40, (uint32_t)nL);
    t_put32(buf + 44, (uint32_t)block);
    t_put32(buf + 48, (uint32_t)qmax);
    for (int j = 0; j < 16; j++) {
      uint32_t u;
      memcpy(&u, &I0.iso[j], 4);
      t_put32(buf + 56 + 4 * j, u);
    }
    t_put64(buf + 120, off);
    if (out_bytes) *out_bytes = off;
    if (!out || cap < off) rc = ORC_E_CAPACITY;
    else memcpy(out, buf, off);
  }
  free(y); free(r); free(rr); free(s); free(cidx); free(cval); free(buf);
  return rc;
}

int orc_tiers_info(const uint8_t *in, uint64_t n, int *T, double *bounds, uint64_t *total) {
  if (n < T_DATA || t_get32(in) != T_MAGIC || t_get32(in + 4) != T_VERSION) return ORC_E_CORRUPT;
  const int t = (int)t_get32(in + 8);
  if (t < 1 || t > ORC_MAX_TIERS) return ORC_E_CORRUPT;
  *T = t;
  for (int k = 0; k < t; k++) bounds[k] = t_getd(in + T_HEAD + T_REC * k);
  *total = t_get64(in + 120);
  return *total <= n ? ORC_OK : ORC_E_CORRUPT;
}

int orc_tiers_decompress(const uint8_t *in, uint64_t n, double eb, float *out, int *tier_used) {
  int T;
  double bounds[ORC_MAX_TIERS];
  uint64_t total;
  int rc = orc_tiers_info(in, n, &T, bounds, &total);
  if (rc) return rc;
  int use = -1;
  for (int t = 0; t < T; t++)
    if (bounds[t] <= eb) { use = t; break; }
  if (use < 0) return ORC_E_ACCURACY;
  int64_t dims[3];
  for (int a = 0; a < 3; a++) dims[a] = (int64_t)t_get64(in + 16 + 8 * a);
  const uint64_t N = (uint64_t)dims[0] * (uint64_t)dims[1] * (uint64_t)dims[2];
  float *rr = (float *)malloc(sizeof(float) * N);
  if (!rr) return ORC_E_NOMEM;
  for (int t = 0; t <= use && rc == ORC_OK; t++) {
    const uint8_t *rec = in + T_HEAD + T_REC * t;
    const uint64_t so = t_get64(rec + 8), sn = t_get64(rec + 16), nc = t_get64(rec + 24);
    const uint64_t io = t_get64(rec + 32), vo = t_get64(rec + 40);
    if (so + sn > total || io + 8 * nc > total || vo + 4 * nc > total) { rc = ORC_E_CORRUPT; break; }
    if (t == 0) {
      rc = orc_decompress(in + so, sn, 0, bounds[0], out);
    } else {
      rc = orc_decompress(in + so, sn, 0, bounds[t], rr);
      if (rc) break;
      for (uint64_t i = 0; i < N; i++) out[i] = out[i] + rr[i];
      for (uint64_t j = 0; j < nc; j++) {
        const uint64_t i = t_get64(in + io + 8 * j);
        if (i >= N) { rc = ORC_E_CORRUPT; break; }
        uint32_t u = t_get32(in + vo + 4 * j);
        memcpy(&out[i], &u, 4);
      }
    }
  }
  free(rr);
  if (rc == ORC_OK && tier_used) *tier_used = use;
  return rc;
}
