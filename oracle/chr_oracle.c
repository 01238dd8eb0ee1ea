/*
 * chr_oracle.c -- CPU oracle for the CHR hot path and marching cubes.
 *
 * TEST INFRASTRUCTURE ONLY: the reference that the GPU library is checked
 * against.  It is loaded only by the tests, the smoke check and the CPU
 * baseline of the benchmark.  It shares no code with the GPU library.
 *
 * The oracle computes ONE global hierarchy, level by level from the coarsest,
 * visiting the points of a level in plain lexicographic order.  There is no
 * blocking, fusion or reordering in the arithmetic; blocks appear only when
 * the finished per-point results are written into the stream, and when a
 * stream is decoded (each closed block on its own, which is what makes the
 * blocks independent).
 *
 * Built with -O2 -ffp-contract=off and without fast-math, so every float
 * operation below is one IEEE binary32 operation rounded to nearest-even.
 */
#include "chr_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAGIC 0x31524843u /* "CHR1" */
#define VERSION 1u
#define HEADER_BYTES 256
#define QMAX_LIMIT 32767

/* ------------------------------------------------------------------------ */
/* little helpers                                                           */
/* ------------------------------------------------------------------------ */

static uint32_t f2u(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }
static float u2f(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }

static void put32(uint8_t *p, uint32_t v) { for (int i = 0; i < 4; i++) p[i] = (uint8_t)(v >> (8 * i)); }
static void put64(uint8_t *p, uint64_t v) { for (int i = 0; i < 8; i++) p[i] = (uint8_t)(v >> (8 * i)); }
static uint32_t get32(const uint8_t *p) { uint32_t v = 0; for (int i = 0; i < 4; i++) v |= (uint32_t)p[i] << (8 * i); return v; }
static uint64_t get64(const uint8_t *p) { uint64_t v = 0; for (int i = 0; i < 8; i++) v |= (uint64_t)p[i] << (8 * i); return v; }
static void putf(uint8_t *p, float f) { put32(p, f2u(f)); }
static float getf(const uint8_t *p) { return u2f(get32(p)); }
static void putd(uint8_t *p, double d) { uint64_t u; memcpy(&u, &d, 8); put64(p, u); }
static double getd(const uint8_t *p) { uint64_t u = get64(p); double d; memcpy(&d, &u, 8); return d; }

static size_t pad8(size_t n) { return (n + 7) & ~(size_t)7; }

/* a < b in the total order of finite binary32 values that puts -0 below +0,
 * so the minimum and maximum of a set are unique bit patterns. */
static int lt_total(float a, float b) {
  if (a != b) return a < b;
  return signbit(a) && !signbit(b);
}

/* MurmurHash3's 32-bit finalizer (a bijection on 32-bit words). */
static uint32_t fmix32(uint32_t h) {
  h ^= h >> 16; h *= 0x85ebca6bu; h ^= h >> 13; h *= 0xc2b2ae35u; h ^= h >> 16;
  return h;
}

/* Stream checksum of a byte range whose length is a multiple of 4: the sum
 * (mod 2^32) of fmix32(word_j XOR j*0x9E3779B9) over its little-endian 32-bit
 * words.  Changing any single word changes the sum. */
static uint32_t checksum(const uint8_t *p, size_t nbytes) {
  uint32_t s = 0;
  for (size_t j = 0; j < nbytes / 4; j++)
    s += fmix32(get32(p + 4 * j) ^ (uint32_t)((uint32_t)j * 0x9E3779B9u));
  return s;
}

static int64_t idx3(const int64_t d[3], int64_t z, int64_t y, int64_t x) {
  return (z * d[1] + y) * d[2] + x;
}

/* ------------------------------------------------------------------------ */
/* hierarchy (reading R4)                                                   */
/* ------------------------------------------------------------------------ */

static int tz(int64_t c) { int t = 0; while (!(c & 1)) { c >>= 1; t++; } return t; }

/* Level of a point: the number of trailing zero bits shared by all three
 * coordinates, capped at the top level nL-1 (a zero coordinate imposes no
 * limit).  Top-level points (multiples of 2^(nL-1)) are the anchors; a point
 * of level l < nL-1 lies on the 2^l grid but not on the 2^(l+1) grid. */
int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

int orc_level_of(int64_t x, int64_t y, int64_t z, int nL) {
  int lv = nL - 1;
  if (x && tz(x) < lv) lv = tz(x);
  if (y && tz(y) < lv) lv = tz(y);
  if (z && tz(z) < lv) lv = tz(z);
  return lv;
}

/* ------------------------------------------------------------------------ */
/* prediction (reading R6)                                                  */
/* ------------------------------------------------------------------------ */

static float avg2(float a, float b) {
  float s = a + b;
  return s * 0.5f;
}

/* Prediction of a non-anchor point (x,y,z) of level l (h = 2^l) from its
 * parents on the 2h grid, read from array a with extents e[] = {ez,ey,ex}.
 * Along every axis where coordinate/h is odd the parents are at -h and +h;
 * when +h falls outside the array the lower parent is used alone.  Averages
 * are taken along x first, then y, then z; avg(a,b) = (a+b)*0.5 in binary32.
 * Anchors are predicted as 0 by the caller. */
static float predict_in(const float *a, const int64_t e[3], int64_t x, int64_t y,
                        int64_t z, int64_t h) {
  int64_t xs[2], ys[2], zs[2];
  int nxp = 1, nyp = 1, nzp = 1;
  xs[0] = xs[1] = x; ys[0] = ys[1] = y; zs[0] = zs[1] = z;
  if ((x / h) & 1) { xs[0] = x - h; xs[1] = x + h; nxp = (x + h < e[2]) ? 2 : 1; }
  if ((y / h) & 1) { ys[0] = y - h; ys[1] = y + h; nyp = (y + h < e[1]) ? 2 : 1; }
  if ((z / h) & 1) { zs[0] = z - h; zs[1] = z + h; nzp = (z + h < e[0]) ? 2 : 1; }
  float vy[2] = {0.f, 0.f};
  for (int iz = 0; iz < nzp; iz++) {
    float vx[2] = {0.f, 0.f};
    for (int iy = 0; iy < nyp; iy++) {
      float v0 = a[idx3(e, zs[iz], ys[iy], xs[0])];
      vx[iy] = (nxp == 2) ? avg2(v0, a[idx3(e, zs[iz], ys[iy], xs[1])]) : v0;
    }
    vy[iz] = (nyp == 2) ? avg2(vx[0], vx[1]) : vx[0];
  }
  return (nzp == 2) ? avg2(vy[0], vy[1]) : vy[0];
}

float orc_predict(const float *xr, const int64_t dims[3], int64_t x, int64_t y,
                  int64_t z, int level, int nL) {
  if (level >= nL - 1) return 0.0f;
  return predict_in(xr, dims, x, y, z, (int64_t)1 << level);
}

/* ------------------------------------------------------------------------ */
/* quantization (reading R7)                                                */
/* ------------------------------------------------------------------------ */

typedef struct {
  double e;
  float inv, step;
  int qmax;
  int lossless;
} quant_t;

/* inv = 1/(2e) and step = 2e are computed in double and rounded to binary32
 * once.  e = 0 (or a step that rounds to 0 or overflows) selects the
 * lossless mode: every code is 0, the reconstruction is the prediction, and a
 * value is stored exactly unless the prediction already equals it bit for bit. */
static void quant_setup(double e, int qmax, quant_t *Q) {
  Q->e = e;
  Q->qmax = qmax;
  Q->inv = 0.f;
  Q->step = 0.f;
  if (e > 0) {
    Q->inv = (float)(1.0 / (2.0 * e));
    Q->step = (float)(2.0 * e);
  }
  Q->lossless = !(e > 0) || Q->step == 0.0f || !isfinite(Q->step);
}

static void quantize_q(float x, float p, const quant_t *Q, int32_t *q, int *O, float *xr) {
  if (Q->lossless) {
    *q = 0;
    *xr = p;
    *O = f2u(p) != f2u(x);
    return;
  }
  float d = x - p;
  float qf = rintf(d * Q->inv); /* round half to even */
  if (!(fabsf(qf) <= (float)Q->qmax)) { /* also catches NaN and infinities */
    *q = 0; *O = 1; *xr = p;
    return;
  }
  float r = qf * Q->step;
  float xq = p + r;
  *q = (int32_t)qf;
  *xr = xq;
  *O = !(fabs((double)xq - (double)x) <= Q->e);
}

void orc_quantize(float x, float p, double e, int qmax, int32_t *q, int *outlier, float *xr) {
  quant_t Q;
  quant_setup(e, qmax, &Q);
  quantize_q(x, p, &Q, q, outlier, xr);
}

/* ------------------------------------------------------------------------ */
/* topology check (Sec. II.B; reading R2)                                   */
/* ------------------------------------------------------------------------ */

/* A vertex value v lies below isovalue k when v < k (reading R1).  With the
 * candidates sorted ascending, the count of k_j <= v determines every one of
 * the K below/not-below bits of the vertex at once. */
int orc_rank(float v, const float *iso, int n_iso) {
  int r = 0;
  for (int j = 0; j < n_iso; j++) r += (iso[j] <= v);
  return r;
}

/* ------------------------------------------------------------------------ */
/* closed blocks (reading R5) and section order                             */
/* ------------------------------------------------------------------------ */

static int64_t nblk_axis(int64_t n, int64_t B) {
  int64_t cells = n - 1;
  if (cells <= 0) return 1;
  return (cells + B - 1) / B;
}

/* Closed extent of block (bz,by,bx): cells [o, o+B) along each axis, points
 * [o, min(o+B, n-1)]. */
static void block_extent(const int64_t dims[3], int64_t B, const int64_t bidx[3],
                         int64_t o[3], int64_t hi[3]) {
  for (int a = 0; a < 3; a++) {
    o[a] = bidx[a] * B;
    hi[a] = o[a] + B;
    if (hi[a] > dims[a] - 1) hi[a] = dims[a] - 1;
  }
}

/* Points of level l in a closed block, lexicographic (z,y,x).  Coordinates
 * are written to pts (3 per point, z,y,x) when pts != NULL. */
static int64_t section_points(const int64_t o[3], const int64_t hi[3], int l, int nL,
                              int64_t *pts) {
  int64_t h = (int64_t)1 << l;
  int64_t n = 0;
  for (int64_t z = o[0]; z <= hi[0]; z += h)
    for (int64_t y = o[1]; y <= hi[1]; y += h)
      for (int64_t x = o[2]; x <= hi[2]; x += h)
        if (orc_level_of(x, y, z, nL) == l) {
          if (pts) { pts[3 * n] = z; pts[3 * n + 1] = y; pts[3 * n + 2] = x; }
          n++;
        }
  return n;
}

/* ------------------------------------------------------------------------ */
/* differentiated error control (Sec. II.A, reading R19)                    */
/* ------------------------------------------------------------------------ */

/* A block is active when the input on its closed extent crosses a candidate
 * isovalue: min < k <= max for some candidate k (with the bit convention of
 * R1 a cell has a crossing iff one corner lies below k and another does
 * not, and a connected extent holding values on both sides has such a cell). */
static void block_activity(const float *x, const int64_t d[3], int64_t B, const int64_t nb[3],
                           const float *iso, int K, uint8_t *act) {
  int64_t nblocks = nb[0] * nb[1] * nb[2];
  for (int64_t b = 0; b < nblocks; b++) {
    int64_t bi[3] = {b / (nb[1] * nb[2]), (b / nb[2]) % nb[1], b % nb[2]}, o[3], hi[3];
    block_extent(d, B, bi, o, hi);
    float mn = x[idx3(d, o[0], o[1], o[2])], mx = mn;
    for (int64_t z = o[0]; z <= hi[0]; z++)
      for (int64_t y = o[1]; y <= hi[1]; y++)
        for (int64_t xx = o[2]; xx <= hi[2]; xx++) {
          float v = x[idx3(d, z, y, xx)];
          if (v < mn) mn = v;
          if (v > mx) mx = v;
        }
    act[b] = 0;
    for (int j = 0; j < K; j++)
      if (mn < iso[j] && iso[j] <= mx) act[b] = 1;
  }
}

/* Blocks along one axis whose closed extent contains coordinate p: c0..c1
 * (two when p is on the face between them). */
static void axis_blocks(int64_t p, int64_t B, int64_t nb, int64_t *c0, int64_t *c1) {
  int64_t c = p / B;
  *c1 = c < nb ? c : nb - 1;
  *c0 = (p % B == 0 && c > 0 && c - 1 < *c1) ? c - 1 : *c1;
}

/* A point takes the near bound when any block whose closed extent contains
 * it is active.  Points shared by blocks so get one bound (their values are
 * the same in every block), and both ends of every crossing edge of a
 * candidate isovalue lie in an active block. */
static int point_near(const uint8_t *act, const int64_t nb[3], int64_t B, int64_t z, int64_t y, int64_t x) {
  int64_t lo[3], hi[3];
  axis_blocks(z, B, nb[0], &lo[0], &hi[0]);
  axis_blocks(y, B, nb[1], &lo[1], &hi[1]);
  axis_blocks(x, B, nb[2], &lo[2], &hi[2]);
  for (int64_t a = lo[0]; a <= hi[0]; a++)
    for (int64_t b = lo[1]; b <= hi[1]; b++)
      for (int64_t c = lo[2]; c <= hi[2]; c++)
        if (act[(a * nb[1] + b) * nb[2] + c]) return 1;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* block merging before compression (Sec. II.A, third step; reading R22)    */
/* ------------------------------------------------------------------------ */

/* Index signature of every block: bit j set when the input on the block's
 * closed extent crosses candidate j (min < k_j <= max).  Blocks with equal
 * signatures answer every query for a candidate isovalue alike. */
static void block_signatures(const float *x, const int64_t d[3], int64_t B, const int64_t nb[3],
                             const float *iso, int K, uint32_t *sig) {
  int64_t nblocks = nb[0] * nb[1] * nb[2];
  for (int64_t b = 0; b < nblocks; b++) {
    int64_t bi[3] = {b / (nb[1] * nb[2]), (b / nb[2]) % nb[1], b % nb[2]}, o[3], hi[3];
    block_extent(d, B, bi, o, hi);
    float mn = x[idx3(d, o[0], o[1], o[2])], mx = mn;
    for (int64_t z = o[0]; z <= hi[0]; z++)
      for (int64_t y = o[1]; y <= hi[1]; y++)
        for (int64_t xx = o[2]; xx <= hi[2]; xx++) {
          float v = x[idx3(d, z, y, xx)];
          if (v < mn) mn = v;
          if (v > mx) mx = v;
        }
    sig[b] = 0;
    for (int j = 0; j < K; j++)
      if (mn < iso[j] && iso[j] <= mx) sig[b] |= 1u << j;
  }
}

/* Greedy merging into rectangular units of at most M blocks per axis: the
 * blocks are visited in lexicographic (z, y, x) order; an unassigned block
 * starts a unit, which grows along x while the next block is unassigned and
 * has the same signature, then along y while the whole next row of the unit
 * qualifies, then along z while the whole next plane does.  Units are
 * numbered in the order they start.  box[8u .. 8u+5] = first block and one
 * past the last block of unit u along z, y, x (box[8u+6..7] = 0).  Returns
 * the number of units; M = 1 gives one unit per block. */
static int64_t merge_units(const uint32_t *sig, const int64_t nb[3], int M, uint32_t *box, int64_t *owner) {
  int64_t nblocks = nb[0] * nb[1] * nb[2], U = 0;
  for (int64_t b = 0; b < nblocks; b++) owner[b] = -1;
#define BLK(z, y, x) (((z) * nb[1] + (y)) * nb[2] + (x))
  for (int64_t z0 = 0; z0 < nb[0]; z0++)
    for (int64_t y0 = 0; y0 < nb[1]; y0++)
      for (int64_t x0 = 0; x0 < nb[2]; x0++) {
        if (owner[BLK(z0, y0, x0)] >= 0) continue;
        uint32_t g = sig[BLK(z0, y0, x0)];
        int64_t ex = 1, ey = 1, ez = 1;
        while (ex < M && x0 + ex < nb[2] && owner[BLK(z0, y0, x0 + ex)] < 0 && sig[BLK(z0, y0, x0 + ex)] == g) ex++;
        for (;;) {
          if (ey >= M || y0 + ey >= nb[1]) break;
          int ok = 1;
          for (int64_t x = x0; x < x0 + ex && ok; x++)
            ok = owner[BLK(z0, y0 + ey, x)] < 0 && sig[BLK(z0, y0 + ey, x)] == g;
          if (!ok) break;
          ey++;
        }
        for (;;) {
          if (ez >= M || z0 + ez >= nb[0]) break;
          int ok = 1;
          for (int64_t y = y0; y < y0 + ey && ok; y++)
            for (int64_t x = x0; x < x0 + ex && ok; x++)
              ok = owner[BLK(z0 + ez, y, x)] < 0 && sig[BLK(z0 + ez, y, x)] == g;
          if (!ok) break;
          ez++;
        }
        for (int64_t z = z0; z < z0 + ez; z++)
          for (int64_t y = y0; y < y0 + ey; y++)
            for (int64_t x = x0; x < x0 + ex; x++) owner[BLK(z, y, x)] = U;
        uint32_t *e = box + 8 * U;
        e[0] = (uint32_t)z0; e[1] = (uint32_t)y0; e[2] = (uint32_t)x0;
        e[3] = (uint32_t)(z0 + ez); e[4] = (uint32_t)(y0 + ey); e[5] = (uint32_t)(x0 + ex);
        e[6] = e[7] = 0;
        U++;
      }
#undef BLK
  return U;
}

/* Closed extent of a unit of blocks b0 .. b1 - 1 per axis (z, y, x): points
 * [b0 B, min(b1 B, n - 1)]. */
static void unit_extent_of(const int64_t dims[3], int64_t B, const uint32_t *e, int64_t o[3], int64_t hi[3]) {
  for (int a = 0; a < 3; a++) {
    o[a] = (int64_t)e[a] * B;
    hi[a] = (int64_t)e[3 + a] * B;
    if (hi[a] > dims[a] - 1) hi[a] = dims[a] - 1;
  }
}

/* ------------------------------------------------------------------------ */
/* section encoding                                                         */
/* ------------------------------------------------------------------------ */

static uint32_t zigzag(int32_t q) { return ((uint32_t)q << 1) ^ (uint32_t)(q >> 31); }
static int32_t unzigzag(uint32_t z) { return (int32_t)(z >> 1) ^ -(int32_t)(z & 1); }
static int bitlen(uint32_t v) { int w = 0; while (v) { w++; v >>= 1; } return w; }

/* Size in bytes of a section given its totals. */
static size_t section_size(int64_t npts, uint64_t W, uint64_t NE, uint64_t NX) {
  int64_t nch = (npts + 63) / 64;
  int64_t ntile = (nch + 63) / 64;
  return 16 + pad8(12 * (size_t)ntile) + pad8((size_t)nch) + 8 * W + 8 * NE + pad8(4 * NX);
}

/* Encodes the n points (codes q, exact flags ef, original values xv) of one
 * section into out (if non-NULL); returns the byte size.  Layout:
 *   u32 npts, u32 W, u32 NE, u32 NX
 *   tile table: per 64 chunks {W, NE, NX before the tile}, padded to 8
 *   chunk headers: u8 per chunk (bits 0-4 width w, bit 7 has-exact), pad 8
 *   payload: per chunk w u64 words; code of lane i at bits [i*w, (i+1)*w)
 *   exact masks: u64 per chunk that has exact values (bit i = lane i)
 *   exact values: binary32 bits, chunk order then lane order, pad 8 */
static size_t encode_section(int64_t n, const int32_t *q, const uint8_t *ef,
                             const float *xv, uint8_t *out) {
  int64_t nch = (n + 63) / 64, ntile = (nch + 63) / 64;
  uint64_t W = 0, NE = 0, NX = 0;
  for (int64_t c = 0; c < nch; c++) {
    uint32_t orv = 0;
    int anyE = 0;
    for (int64_t i = 64 * c; i < n && i < 64 * c + 64; i++) {
      if (ef[i]) { anyE = 1; NX++; } else orv |= zigzag(q[i]);
    }
    W += (uint64_t)bitlen(orv);
    NE += (uint64_t)anyE;
  }
  size_t bytes = section_size(n, W, NE, NX);
  if (!out) return bytes;
  memset(out, 0, bytes);
  size_t o_tile = 16, o_hdr = o_tile + pad8(12 * (size_t)ntile), o_pay = o_hdr + pad8((size_t)nch);
  size_t o_msk = o_pay + 8 * W, o_ex = o_msk + 8 * NE;
  put32(out, (uint32_t)n); put32(out + 4, (uint32_t)W); put32(out + 8, (uint32_t)NE); put32(out + 12, (uint32_t)NX);
  uint64_t w_run = 0, e_run = 0, x_run = 0;
  for (int64_t c = 0; c < nch; c++) {
    if (c % 64 == 0) {
      uint8_t *t = out + o_tile + 12 * (size_t)(c / 64);
      put32(t, (uint32_t)w_run); put32(t + 4, (uint32_t)e_run); put32(t + 8, (uint32_t)x_run);
    }
    uint32_t zc[64];
    uint64_t emask = 0;
    uint32_t orv = 0;
    for (int i = 0; i < 64; i++) {
      int64_t j = 64 * c + i;
      zc[i] = 0;
      if (j < n) {
        if (ef[j]) emask |= (uint64_t)1 << i;
        else zc[i] = zigzag(q[j]);
      }
      orv |= zc[i];
    }
    int w = bitlen(orv);
    out[o_hdr + c] = (uint8_t)(w | (emask ? 0x80 : 0));
    uint8_t *pay = out + o_pay + 8 * w_run;
    for (int i = 0; i < 64; i++)
      for (int b = 0; b < w; b++)
        if ((zc[i] >> b) & 1) {
          int64_t bit = (int64_t)i * w + b;
          pay[bit / 8] |= (uint8_t)(1u << (bit % 8));
        }
    w_run += (uint64_t)w;
    if (emask) {
      put64(out + o_msk + 8 * e_run, emask);
      e_run++;
      for (int i = 0; i < 64; i++)
        if ((emask >> i) & 1) { putf(out + o_ex + 4 * x_run, xv[64 * c + i]); x_run++; }
    }
  }
  return bytes;
}

/* ------------------------------------------------------------------------ */
/* compression                                                              */
/* ------------------------------------------------------------------------ */

static int cmp_float(const void *a, const void *b) {
  float fa = *(const float *)a, fb = *(const float *)b;
  return (fa > fb) - (fa < fb);
}

/* Sorts and de-duplicates the candidate isovalues (reading R16). */
static int prepare_iso(const float *iso, int n_iso, float out[16]) {
  if (n_iso < 0 || n_iso > 16) return -1;
  float t[16];
  for (int j = 0; j < n_iso; j++) {
    if (!isfinite(iso[j])) return -1;
    t[j] = iso[j];
  }
  qsort(t, (size_t)n_iso, sizeof(float), cmp_float);
  int k = 0;
  for (int j = 0; j < n_iso; j++)
    if (k == 0 || t[j] != out[k - 1]) out[k++] = t[j];
  for (int j = k; j < 16; j++) out[j] = 0.f;
  return k;
}

size_t orc_compress_bound_merged(const int64_t dims[3], int nL, int block, int merge) {
  /* a unit's sections are no larger than its blocks' together (fewer points,
   * fewer section overheads); each unit adds a 32-byte box entry */
  size_t t = orc_compress_bound(dims, nL, block);
  if (merge > 1) {
    int64_t nblocks = nblk_axis(dims[0], block) * nblk_axis(dims[1], block) * nblk_axis(dims[2], block);
    t += 32 * (size_t)nblocks;
  }
  return t;
}

size_t orc_compress_bound(const int64_t dims[3], int nL, int block) {
  int64_t nb[3];
  for (int a = 0; a < 3; a++) nb[a] = nblk_axis(dims[a], block);
  int64_t nblocks = nb[0] * nb[1] * nb[2];
  size_t total = HEADER_BYTES + 16 * (size_t)nblocks * (size_t)nL + 16 * (size_t)nblocks;
  for (int64_t bz = 0; bz < nb[0]; bz++)
    for (int64_t by = 0; by < nb[1]; by++)
      for (int64_t bx = 0; bx < nb[2]; bx++) {
        int64_t bi[3] = {bz, by, bx}, o[3], hi[3];
        block_extent(dims, block, bi, o, hi);
        for (int l = nL - 1; l >= 0; l--) {
          int64_t n = section_points(o, hi, l, nL, NULL);
          int64_t nch = (n + 63) / 64;
          total += section_size(n, 16 * (uint64_t)nch, (uint64_t)nch, (uint64_t)n);
        }
      }
  return total;
}

static int check_params(const int64_t dims[3], int nL, int block, int qmax) {
  if (nL < 1 || nL > 16) return -1;
  for (int a = 0; a < 3; a++)
    if (dims[a] < 1 || dims[a] > ((int64_t)1 << 30)) return -1;
  int64_t S = (int64_t)1 << (nL - 1);
  if (block < 1 || block % S) return -1;
  if (qmax < 1 || qmax > QMAX_LIMIT) return -1;
  return 0;
}

/* Largest unit extent (in points) of merged blocks must stay below 2^31
 * points, as a block's closed extent does. */
static int merge_ok(const int64_t dims[3], int block, int merge) {
  if (merge < 0 || merge > 16) return 0;
  if (merge <= 1) return 1;
  double pts = 1;
  for (int a = 0; a < 3; a++) {
    int64_t e = (int64_t)merge * block;
    if (e > dims[a] - 1) e = dims[a] - 1;
    pts *= (double)(e + 1);
  }
  return pts < 2147483648.0;
}

int orc_compress(const float *x, const int64_t dims[3], double error_bound, double error_bound_far,
                 const float *iso_in, int n_iso_in, int nL, int block, int qmax,
                 int32_t *q_out, uint8_t *flags_out, float *xr_out,
                 uint8_t *stream, size_t cap, size_t *stream_bytes) {
  return orc_compress_merged(x, dims, error_bound, error_bound_far, iso_in, n_iso_in, nL, block, qmax, 1, q_out,
                             flags_out, xr_out, stream, cap, stream_bytes);
}

int orc_compress_merged(const float *x, const int64_t dims[3], double error_bound, double error_bound_far,
                        const float *iso_in, int n_iso_in, int nL, int block, int qmax, int merge,
                        int32_t *q_out, uint8_t *flags_out, float *xr_out,
                        uint8_t *stream, size_t cap, size_t *stream_bytes) {
  if (check_params(dims, nL, block, qmax)) return ORC_E_INVAL;
  if (!merge_ok(dims, block, merge)) return ORC_E_INVAL;
  /* merging is not combined with differentiated error control */
  if (merge > 1 && error_bound_far != 0) return ORC_E_INVAL;
  if (!(error_bound >= 0) || !isfinite(error_bound)) return ORC_E_INVAL;
  /* far bound: 0 for one bound everywhere, else finite and >= error_bound */
  if (error_bound_far != 0 && !(error_bound_far >= error_bound && isfinite(error_bound_far))) return ORC_E_INVAL;
  const int diff = error_bound_far != 0;
  float iso[16];
  int K = prepare_iso(iso_in, n_iso_in, iso);
  if (K < 0) return ORC_E_INVAL;
  int64_t N = dims[0] * dims[1] * dims[2];
  for (int64_t i = 0; i < N; i++)
    if (!isfinite(x[i])) return ORC_E_INVAL; /* reading R15 */
  quant_t Q, Qf;
  quant_setup(error_bound, qmax, &Q);
  quant_setup(diff ? error_bound_far : 0.0, qmax, &Qf);
  int64_t nb[3];
  for (int a = 0; a < 3; a++) nb[a] = nblk_axis(dims[a], block);
  int64_t nblocks = nb[0] * nb[1] * nb[2];

  float *xr = (float *)malloc(sizeof(float) * (size_t)N);
  int32_t *q = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
  uint8_t *fl = (uint8_t *)malloc((size_t)N);
  uint8_t *act = (uint8_t *)calloc((size_t)nblocks, 1);
  uint32_t *sig = (uint32_t *)calloc((size_t)nblocks, sizeof(uint32_t));
  uint32_t *box = (uint32_t *)malloc(sizeof(uint32_t) * 8 * (size_t)nblocks);
  int64_t *owner = (int64_t *)malloc(sizeof(int64_t) * (size_t)nblocks);
  if (!xr || !q || !fl || !act || !sig || !box || !owner) {
    free(xr); free(q); free(fl); free(act); free(sig); free(box); free(owner);
    return ORC_E_NOMEM;
  }
  if (diff) block_activity(x, dims, block, nb, iso, K, act);
  /* storage units: the blocks themselves, or merged rectangles of blocks
   * with equal index signatures (reading R22) */
  const int merged = merge > 1;
  if (merged) block_signatures(x, dims, block, nb, iso, K, sig);
  const int64_t U = merge_units(sig, nb, merged ? merge : 1, box, owner);
  free(sig); free(owner);
  uint32_t mb[3] = {0, 0, 0};
  for (int64_t u = 0; u < U; u++)
    for (int a = 0; a < 3; a++)
      if (box[8 * u + 3 + a] - box[8 * u + a] > mb[a]) mb[a] = box[8 * u + 3 + a] - box[8 * u + a];

  /* Levels from the coarsest; the points of one level depend only on
   * reconstructed values of coarser levels, so their order is immaterial. */
  uint64_t nO = 0, nC = 0;
  for (int l = nL - 1; l >= 0; l--) {
    int64_t h = (int64_t)1 << l;
#pragma omp parallel for schedule(static) reduction(+ : nO, nC)
    for (int64_t z = 0; z < dims[0]; z += h)
      for (int64_t y = 0; y < dims[1]; y += h)
        for (int64_t xx = 0; xx < dims[2]; xx += h) {
          if (orc_level_of(xx, y, z, nL) != l) continue;
          int64_t i = idx3(dims, z, y, xx);
          float v = x[i];
          /* prediction (R6) and quantization (R7) */
          float p = (l == nL - 1) ? 0.0f : predict_in(xr, dims, xx, y, z, h);
          int32_t code; int O; float r;
          const quant_t *Qp = (diff && !point_near(act, nb, block, z, y, xx)) ? &Qf : &Q;
          quantize_q(v, p, Qp, &code, &O, &r);
          /* topology check on the candidate reconstruction (R2, R8): the
           * vertex must stay on the same side of every candidate isovalue */
          int C = 0;
          if (!O) C = orc_rank(v, iso, K) != orc_rank(r, iso, K);
          /* correction (R3): an offending vertex is stored exactly, so its
           * error is 0, below every distance d0, d1 of Sec. II.B */
          if (O || C) { r = v; code = 0; }
          xr[i] = r;
          q[i] = code;
          fl[i] = (uint8_t)(O | (C << 1));
          nO += (uint64_t)O;
          nC += (uint64_t)C;
        }
  }

  /* stream (reading R9): tables per unit; a merged stream adds the box
   * table of its units after the unit (block) table */
  size_t tab = HEADER_BYTES, btab = tab + 16 * (size_t)U * (size_t)nL;
  size_t xtab = btab + 16 * (size_t)U;
  size_t payload = xtab + (merged ? 32 * (size_t)U : 0);

  /* pass 1: sizes; pass 2: write */
  size_t total = payload;
  int64_t maxn = 0;
  for (int64_t b = 0; b < U; b++) {
    int64_t o[3], hi[3];
    unit_extent_of(dims, block, box + 8 * b, o, hi);
    for (int l = nL - 1; l >= 0; l--) {
      int64_t n = section_points(o, hi, l, nL, NULL);
      if (n > maxn) maxn = n;
    }
  }
  int64_t *pts = (int64_t *)malloc(sizeof(int64_t) * 3 * (size_t)(maxn ? maxn : 1));
  int32_t *sq = (int32_t *)malloc(sizeof(int32_t) * (size_t)(maxn ? maxn : 1));
  uint8_t *se = (uint8_t *)malloc((size_t)(maxn ? maxn : 1));
  float *sx = (float *)malloc(sizeof(float) * (size_t)(maxn ? maxn : 1));
  if (!pts || !sq || !se || !sx) {
    free(pts); free(sq); free(se); free(sx); free(xr); free(q); free(fl); free(act); free(box);
    return ORC_E_NOMEM;
  }
  for (int pass = 0; pass < 2; pass++) {
    size_t off = payload;
    for (int64_t b = 0; b < U; b++) {
      int64_t o[3], hi[3];
      unit_extent_of(dims, block, box + 8 * b, o, hi);
      size_t bstart = off;
      float bmin = INFINITY, bmax = -INFINITY;
      for (int l = nL - 1; l >= 0; l--) {
        int64_t n = section_points(o, hi, l, nL, pts);
        for (int64_t j = 0; j < n; j++) {
          int64_t i = idx3(dims, pts[3 * j], pts[3 * j + 1], pts[3 * j + 2]);
          sq[j] = q[i];
          se[j] = fl[i] != 0;
          sx[j] = x[i];
          if (lt_total(xr[i], bmin)) bmin = xr[i];
          if (lt_total(bmax, xr[i])) bmax = xr[i];
        }
        size_t sz = encode_section(n, sq, se, sx, NULL);
        if (pass == 1) {
          encode_section(n, sq, se, sx, stream + off);
          uint8_t *ent = stream + tab + 16 * ((size_t)b * (size_t)nL + (size_t)(nL - 1 - l));
          put64(ent, off);
          put64(ent + 8, sz);
        }
        off += sz;
      }
      if (pass == 1) {
        uint8_t *be = stream + btab + 16 * (size_t)b;
        putf(be, bmin);
        putf(be + 4, bmax);
        put32(be + 8, checksum(stream + bstart, off - bstart));
        put32(be + 12, diff ? (uint32_t)act[b] : 0u);  /* bit 0: active block (R19) */
        if (merged)
          for (int k = 0; k < 8; k++) put32(stream + xtab + 32 * (size_t)b + 4 * (size_t)k, box[8 * b + k]);
      }
    }
    total = off;
    if (pass == 0) {
      if (stream_bytes) *stream_bytes = total;
      if (!stream || cap < total) {
        free(pts); free(sq); free(se); free(sx); free(xr); free(q); free(fl); free(act); free(box);
        return ORC_E_CAPACITY;
      }
      memset(stream, 0, total);
    }
  }
  free(pts); free(sq); free(se); free(sx); free(box);

  /* header */
  float vmin = INFINITY, vmax = -INFINITY;
  for (int64_t i = 0; i < N; i++) {
    if (lt_total(x[i], vmin)) vmin = x[i];
    if (lt_total(vmax, x[i])) vmax = x[i];
  }
  uint8_t *H = stream;
  put32(H + 0, MAGIC);
  put32(H + 4, VERSION);
  for (int a = 0; a < 3; a++) put64(H + 8 + 8 * a, (uint64_t)dims[a]);
  put32(H + 32, (uint32_t)nL);
  put32(H + 36, (uint32_t)block);
  put32(H + 40, (uint32_t)qmax);
  put32(H + 44, (uint32_t)K);
  putd(H + 48, error_bound);
  putf(H + 56, Q.inv);
  putf(H + 60, Q.step);
  for (int j = 0; j < 16; j++) putf(H + 64 + 4 * j, iso[j]);
  putf(H + 128, vmin);
  putf(H + 132, vmax);
  put64(H + 136, (uint64_t)U);
  for (int a = 0; a < 3; a++) put32(H + 144 + 4 * a, (uint32_t)nb[a]);
  put32(H + 156, (Q.lossless ? 1u : 0u) | (diff ? 2u : 0u) | (diff && Qf.lossless ? 4u : 0u) | (merged ? 8u : 0u));
  put64(H + 160, total);
  put64(H + 168, nO);
  put64(H + 176, nC);
  put64(H + 184, payload);
  if (diff) {
    putd(H + 192, error_bound_far);
    putf(H + 200, Qf.inv);
    putf(H + 204, Qf.step);
  }
  if (merged) {
    put32(H + 208, (uint32_t)merge);
    for (int a = 0; a < 3; a++) put32(H + 212 + 4 * a, mb[a]);
  }
  put32(H + 248, checksum(stream + HEADER_BYTES, payload - HEADER_BYTES));
  put32(H + 252, checksum(H, 252));

  if (q_out) memcpy(q_out, q, sizeof(int32_t) * (size_t)N);
  if (flags_out) memcpy(flags_out, fl, (size_t)N);
  if (xr_out) memcpy(xr_out, xr, sizeof(float) * (size_t)N);
  free(xr); free(q); free(fl); free(act);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* stream reading                                                           */
/* ------------------------------------------------------------------------ */

int orc_stream_info(const uint8_t *s, size_t n, orc_info *I) {
  if (n < HEADER_BYTES) return ORC_E_CORRUPT;
  if (get32(s) != MAGIC || get32(s + 4) != VERSION) return ORC_E_CORRUPT;
  if (checksum(s, 252) != get32(s + 252)) return ORC_E_CORRUPT;
  memset(I, 0, sizeof(*I));
  for (int a = 0; a < 3; a++) I->dims[a] = (int64_t)get64(s + 8 + 8 * a);
  I->levels = (int)get32(s + 32);
  I->block = (int)get32(s + 36);
  I->qmax = (int)get32(s + 40);
  I->n_iso = (int)get32(s + 44);
  I->error_bound = getd(s + 48);
  I->inv = getf(s + 56);
  I->step = getf(s + 60);
  for (int j = 0; j < 16; j++) I->iso[j] = getf(s + 64 + 4 * j);
  I->vmin = getf(s + 128);
  I->vmax = getf(s + 132);
  I->nblocks = (int64_t)get64(s + 136);
  for (int a = 0; a < 3; a++) I->nb[a] = (int)get32(s + 144 + 4 * a);
  I->flags = get32(s + 156);
  I->total_bytes = get64(s + 160);
  I->n_outlier = get64(s + 168);
  I->n_corrected = get64(s + 176);
  I->payload_offset = get64(s + 184);
  I->error_bound_far = getd(s + 192);
  I->inv_far = getf(s + 200);
  I->step_far = getf(s + 204);
  const int merged = (I->flags & 8u) != 0;
  I->merge = merged ? (int)get32(s + 208) : 1;
  for (int a = 0; a < 3; a++) I->mb[a] = merged ? (int)get32(s + 212 + 4 * a) : 1;
  if (I->flags & ~15u) return ORC_E_CORRUPT;
  if ((I->flags & 2u) && !(I->error_bound_far >= I->error_bound && isfinite(I->error_bound_far))) return ORC_E_CORRUPT;
  if (merged && (I->flags & 2u)) return ORC_E_CORRUPT;
  if (check_params(I->dims, I->levels, I->block, I->qmax)) return ORC_E_CORRUPT;
  if (merged && (I->merge < 2 || !merge_ok(I->dims, I->block, I->merge))) return ORC_E_CORRUPT;
  for (int a = 0; a < 3; a++)
    if (I->mb[a] < 1 || I->mb[a] > I->merge || I->nb[a] != nblk_axis(I->dims[a], I->block)) return ORC_E_CORRUPT;
  const int64_t nbt = (int64_t)I->nb[0] * I->nb[1] * I->nb[2];
  if (I->nblocks < 1 || I->nblocks > nbt || (!merged && I->nblocks != nbt)) return ORC_E_CORRUPT;
  if (I->n_iso < 0 || I->n_iso > 16) return ORC_E_CORRUPT;
  if (I->total_bytes > n) return ORC_E_CORRUPT;
  if (I->payload_offset != HEADER_BYTES + 16 * (uint64_t)I->nblocks * (uint64_t)I->levels + 16 * (uint64_t)I->nblocks +
                               (merged ? 32 * (uint64_t)I->nblocks : 0))
    return ORC_E_CORRUPT;
  if (I->payload_offset > I->total_bytes) return ORC_E_CORRUPT;
  if (checksum(s + HEADER_BYTES, I->payload_offset - HEADER_BYTES) != get32(s + 248)) return ORC_E_CORRUPT;
  if (merged) {
    /* the units tile the block grid: every block in exactly one unit, none
     * wider than the stored largest extent */
    uint8_t *seen = (uint8_t *)calloc((size_t)nbt, 1);
    if (!seen) return ORC_E_NOMEM;
    const uint8_t *xt = s + HEADER_BYTES + 16 * (size_t)I->nblocks * (size_t)I->levels + 16 * (size_t)I->nblocks;
    int bad = 0;
    for (int64_t u = 0; u < I->nblocks && !bad; u++) {
      uint32_t e[8];
      for (int k = 0; k < 8; k++) e[k] = get32(xt + 32 * (size_t)u + 4 * (size_t)k);
      for (int a = 0; a < 3; a++)
        if (e[a] >= e[3 + a] || e[3 + a] > (uint32_t)I->nb[a] || e[3 + a] - e[a] > (uint32_t)I->mb[a]) bad = 1;
      if (e[6] || e[7]) bad = 1;
      for (uint32_t z = e[0]; z < e[3] && !bad; z++)
        for (uint32_t y = e[1]; y < e[4] && !bad; y++)
          for (uint32_t x = e[2]; x < e[5] && !bad; x++) {
            uint8_t *f = seen + ((int64_t)z * I->nb[1] + y) * I->nb[2] + x;
            if (*f) bad = 1;
            *f = 1;
          }
    }
    for (int64_t b = 0; b < nbt && !bad; b++)
      if (!seen[b]) bad = 1;
    free(seen);
    if (bad) return ORC_E_CORRUPT;
  }
  return ORC_OK;
}

/* Closed extent of storage unit u of a stream (a block, or a merged box). */
static void unit_extent(const uint8_t *s, const orc_info *I, int64_t u, int64_t o[3], int64_t hi[3]) {
  uint32_t e[8];
  if (I->flags & 8u) {
    const uint8_t *xt = s + HEADER_BYTES + 16 * (size_t)I->nblocks * (size_t)I->levels + 16 * (size_t)I->nblocks;
    for (int k = 0; k < 6; k++) e[k] = get32(xt + 32 * (size_t)u + 4 * (size_t)k);
  } else {
    e[0] = (uint32_t)(u / ((int64_t)I->nb[1] * I->nb[2]));
    e[1] = (uint32_t)((u / I->nb[2]) % I->nb[1]);
    e[2] = (uint32_t)(u % I->nb[2]);
    for (int a = 0; a < 3; a++) e[3 + a] = e[a] + 1;
  }
  unit_extent_of(I->dims, I->block, e, o, hi);
}

int orc_stream_verify(const uint8_t *s, size_t n) {
  orc_info I;
  int rc = orc_stream_info(s, n, &I);
  if (rc) return rc;
  size_t tab = HEADER_BYTES, btab = tab + 16 * (size_t)I.nblocks * (size_t)I.levels;
  for (int64_t b = 0; b < I.nblocks; b++) {
    const uint8_t *first = s + tab + 16 * ((size_t)b * (size_t)I.levels);
    const uint8_t *last = s + tab + 16 * ((size_t)b * (size_t)I.levels + (size_t)I.levels - 1);
    uint64_t start = get64(first), end = get64(last) + get64(last + 8);
    if (start > end || end > I.total_bytes) return ORC_E_CORRUPT;
    if (checksum(s + start, end - start) != get32(s + btab + 16 * (size_t)b + 8)) return ORC_E_CORRUPT;
  }
  return ORC_OK;
}

/* Decodes one section into codes q[], exact flags ef[] and exact values xv[]
 * for its n points; checks the tile table against the running totals. */
static int decode_section(const uint8_t *sec, size_t avail, int64_t n, int32_t *q,
                          uint8_t *ef, float *xv) {
  if (avail < 16) return ORC_E_CORRUPT;
  if ((int64_t)get32(sec) != n) return ORC_E_CORRUPT;
  uint64_t W = get32(sec + 4), NE = get32(sec + 8), NX = get32(sec + 12);
  if (section_size(n, W, NE, NX) > avail) return ORC_E_CORRUPT;
  int64_t nch = (n + 63) / 64, ntile = (nch + 63) / 64;
  size_t o_tile = 16, o_hdr = o_tile + pad8(12 * (size_t)ntile), o_pay = o_hdr + pad8((size_t)nch);
  size_t o_msk = o_pay + 8 * W, o_ex = o_msk + 8 * NE;
  uint64_t w_run = 0, e_run = 0, x_run = 0;
  for (int64_t c = 0; c < nch; c++) {
    if (c % 64 == 0) {
      const uint8_t *t = sec + o_tile + 12 * (size_t)(c / 64);
      if (get32(t) != w_run || get32(t + 4) != e_run || get32(t + 8) != x_run) return ORC_E_CORRUPT;
    }
    uint8_t hb = sec[o_hdr + c];
    int w = hb & 31;
    if (w > 16 || (hb & 0x60)) return ORC_E_CORRUPT;
    if (w_run + (uint64_t)w > W) return ORC_E_CORRUPT;
    const uint8_t *pay = sec + o_pay + 8 * w_run;
    uint64_t emask = 0;
    if (hb & 0x80) {
      if (e_run >= NE) return ORC_E_CORRUPT;
      emask = get64(sec + o_msk + 8 * e_run);
      e_run++;
    }
    for (int i = 0; i < 64; i++) {
      int64_t j = 64 * c + i;
      uint32_t zc = 0;
      for (int b = 0; b < w; b++) {
        int64_t bit = (int64_t)i * w + b;
        zc |= (uint32_t)((pay[bit / 8] >> (bit % 8)) & 1) << b;
      }
      if (j >= n) continue;
      ef[j] = (emask >> i) & 1;
      q[j] = unzigzag(zc);
      if (ef[j]) {
        if (x_run >= NX) return ORC_E_CORRUPT;
        xv[j] = getf(sec + o_ex + 4 * x_run);
        x_run++;
      }
    }
    w_run += (uint64_t)w;
  }
  if (w_run != W || e_run != NE || x_run != NX) return ORC_E_CORRUPT;
  return ORC_OK;
}

static const uint8_t *section_at(const uint8_t *s, const orc_info *I, int64_t b, int l,
                                 size_t *avail) {
  const uint8_t *ent = s + HEADER_BYTES + 16 * ((size_t)b * (size_t)I->levels + (size_t)(I->levels - 1 - l));
  uint64_t off = get64(ent), sz = get64(ent + 8);
  if (off < I->payload_offset || off + sz > I->total_bytes || (off & 7)) return NULL;
  *avail = sz;
  return s + off;
}

int orc_stream_codes(const uint8_t *s, size_t n, int32_t *q_out, uint8_t *e_out) {
  orc_info I;
  int rc = orc_stream_info(s, n, &I);
  if (rc) return rc;
  int nL = I.levels;
  int64_t maxn = 0;
  for (int64_t b = 0; b < I.nblocks; b++) {
    int64_t o[3], hi[3];
    unit_extent(s, &I, b, o, hi);
    for (int l = nL - 1; l >= 0; l--) {
      int64_t m = section_points(o, hi, l, nL, NULL);
      if (m > maxn) maxn = m;
    }
  }
  size_t m1 = (size_t)(maxn ? maxn : 1);
  int64_t *pts = (int64_t *)malloc(sizeof(int64_t) * 3 * m1);
  int32_t *sq = (int32_t *)malloc(sizeof(int32_t) * m1);
  uint8_t *se = (uint8_t *)malloc(m1);
  float *sx = (float *)malloc(sizeof(float) * m1);
  if (!pts || !sq || !se || !sx) { free(pts); free(sq); free(se); free(sx); return ORC_E_NOMEM; }
  rc = ORC_OK;
  for (int64_t b = 0; b < I.nblocks && rc == ORC_OK; b++) {
    int64_t o[3], hi[3];
    unit_extent(s, &I, b, o, hi);
    for (int l = nL - 1; l >= 0 && rc == ORC_OK; l--) {
      int64_t m = section_points(o, hi, l, nL, pts);
      size_t avail;
      const uint8_t *sec = section_at(s, &I, b, l, &avail);
      if (!sec) { rc = ORC_E_CORRUPT; break; }
      rc = decode_section(sec, avail, m, sq, se, sx);
      if (rc) break;
      for (int64_t j = 0; j < m; j++) {
        int64_t i = idx3(I.dims, pts[3 * j], pts[3 * j + 1], pts[3 * j + 2]);
        q_out[i] = sq[j];
        e_out[i] = se[j];
      }
    }
  }
  free(pts); free(sq); free(se); free(sx);
  return rc;
}

/* Reconstruction (reading R10).  Every closed block is decoded into a local
 * array of its own extent from its own sections, coarsest level first,
 * exactly mirroring compression: x' = exact value where stored exactly, else
 * prediction + code*step (prediction alone in lossless mode). */
int orc_decompress(const uint8_t *s, size_t n, int level, double eb, float *out) {
  orc_info I;
  int rc = orc_stream_info(s, n, &I);
  if (rc) return rc;
  int nL = I.levels;
  if (level < 0 || level >= nL) return ORC_E_LEVEL;
  const int diff = (I.flags & 2u) != 0;
  /* accuracy: the loosest bound the stream holds */
  if (!(eb >= (diff ? I.error_bound_far : I.error_bound))) return ORC_E_ACCURACY;
  quant_t Q, Qf;
  quant_setup(I.error_bound, I.qmax, &Q);
  quant_setup(diff ? I.error_bound_far : 0.0, I.qmax, &Qf);
  if (f2u(Q.inv) != f2u(I.inv) || f2u(Q.step) != f2u(I.step)) return ORC_E_CORRUPT;
  if (diff && (f2u(Qf.inv) != f2u(I.inv_far) || f2u(Qf.step) != f2u(I.step_far))) return ORC_E_CORRUPT;
  const int64_t nbk[3] = {I.nb[0], I.nb[1], I.nb[2]};
  uint8_t *act = (uint8_t *)calloc((size_t)I.nblocks, 1);
  if (!act) return ORC_E_NOMEM;
  {
    size_t btab = HEADER_BYTES + 16 * (size_t)I.nblocks * (size_t)I.levels;
    for (int64_t b = 0; b < I.nblocks; b++) act[b] = diff && (get32(s + btab + 16 * (size_t)b + 12) & 1u);
  }
  int64_t od[3];
  for (int a = 0; a < 3; a++) od[a] = ((I.dims[a] - 1) >> level) + 1;
  int64_t B = I.block;
  size_t le = 1;  /* points of the largest unit */
  for (int a = 0; a < 3; a++) {
    int64_t e = (int64_t)I.mb[a] * B;
    le *= (size_t)((e < I.dims[a] - 1 ? e : I.dims[a] - 1) + 1);
  }
  float *loc = (float *)malloc(sizeof(float) * le);
  int64_t *pts = (int64_t *)malloc(sizeof(int64_t) * 3 * le);
  int32_t *sq = (int32_t *)malloc(sizeof(int32_t) * le);
  uint8_t *se = (uint8_t *)malloc(le);
  float *sx = (float *)malloc(sizeof(float) * le);
  if (!loc || !pts || !sq || !se || !sx) { free(loc); free(pts); free(sq); free(se); free(sx); free(act); return ORC_E_NOMEM; }
  rc = ORC_OK;
  for (int64_t b = 0; b < I.nblocks && rc == ORC_OK; b++) {
    int64_t o[3], hi[3];
    unit_extent(s, &I, b, o, hi);
    int64_t le3[3] = {hi[0] - o[0] + 1, hi[1] - o[1] + 1, hi[2] - o[2] + 1};
    for (int l = nL - 1; l >= level && rc == ORC_OK; l--) {
      int64_t m = section_points(o, hi, l, nL, pts);
      size_t avail;
      const uint8_t *sec = section_at(s, &I, b, l, &avail);
      if (!sec) { rc = ORC_E_CORRUPT; break; }
      rc = decode_section(sec, avail, m, sq, se, sx);
      if (rc) break;
      int64_t h = (int64_t)1 << l;
      for (int64_t j = 0; j < m; j++) {
        int64_t z = pts[3 * j] - o[0], y = pts[3 * j + 1] - o[1], x = pts[3 * j + 2] - o[2];
        float r;
        if (se[j]) {
          r = sx[j];
        } else {
          float p = (l == nL - 1) ? 0.0f : predict_in(loc, le3, x, y, z, h);
          const quant_t *Qp = (diff && !point_near(act, nbk, B, pts[3 * j], pts[3 * j + 1], pts[3 * j + 2])) ? &Qf : &Q;
          if (Qp->lossless) r = p;
          else { float t = (float)sq[j] * Qp->step; r = p + t; }
        }
        loc[idx3(le3, z, y, x)] = r;
      }
    }
    if (rc) break;
    int64_t hs = (int64_t)1 << level;
    for (int64_t z = o[0]; z <= hi[0]; z += hs)
      for (int64_t y = o[1]; y <= hi[1]; y += hs)
        for (int64_t x = o[2]; x <= hi[2]; x += hs)
          out[idx3(od, z >> level, y >> level, x >> level)] =
              loc[idx3(le3, z - o[0], y - o[1], x - o[2])];
  }
  free(loc); free(pts); free(sq); free(se); free(sx); free(act);
  return rc;
}

int orc_block_index(const uint8_t *s, size_t n, float *mins, float *maxs) {
  orc_info I;
  int rc = orc_stream_info(s, n, &I);
  if (rc) return rc;
  size_t btab = HEADER_BYTES + 16 * (size_t)I.nblocks * (size_t)I.levels;
  for (int64_t b = 0; b < I.nblocks; b++) {
    mins[b] = getf(s + btab + 16 * (size_t)b);
    maxs[b] = getf(s + btab + 16 * (size_t)b + 4);
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* marching cubes (Sec. I; Sec. II.B; readings R1, R11-R13)                 */
/* ------------------------------------------------------------------------ */

/* Cell corners: v = dx + 2dy + 4dz.  Cell edges: 0..3 run along x at
 * (dy,dz) = (0,0),(1,0),(0,1),(1,1); 4..7 along y at (dx,dz) in the same
 * order; 8..11 along z at (dx,dy).  Edge e joins corners lo(e) and hi(e). */
static void edge_corners(int e, int *lo, int *hi) {
  int a = e / 4, i = e % 4, p = i & 1, r = i >> 1;
  int c[3] = {0, 0, 0}; /* dx, dy, dz */
  if (a == 0) { c[1] = p; c[2] = r; }
  if (a == 1) { c[0] = p; c[2] = r; }
  if (a == 2) { c[0] = p; c[1] = r; }
  *lo = c[0] + 2 * c[1] + 4 * c[2];
  c[a] = 1;
  *hi = c[0] + 2 * c[1] + 4 * c[2];
}

static int edge_between(int c0, int c1) {
  for (int e = 0; e < 12; e++) {
    int lo, hi;
    edge_corners(e, &lo, &hi);
    if ((lo == c0 && hi == c1) || (lo == c1 && hi == c0)) return e;
  }
  return -1;
}

/* Table rule (reading R12).  On every face, the crossed edges are paired:
 * two crossed edges form one segment; four crossed edges (below corners on a
 * diagonal) form the two segments that each cut off one below corner.  Every
 * crossed edge then has two neighbours, so the segments form disjoint loops.
 * Each loop is oriented so that its normal (Newell's formula over the edge
 * midpoints) points from below to above, rotated to start at its smallest
 * edge id, and fan-triangulated from there.  Loops are emitted in order of
 * their smallest edge id. */
void orc_mc_table(uint8_t ntri[256], int8_t tri[256][3 * ORC_MC_MAXTRI]) {
  /* faces as corner cycles */
  static const int face[6][4] = {
      {0, 2, 6, 4}, {1, 3, 7, 5}, /* x = 0, x = 1 */
      {0, 1, 5, 4}, {2, 3, 7, 6}, /* y = 0, y = 1 */
      {0, 1, 3, 2}, {4, 5, 7, 6}  /* z = 0, z = 1 */
  };
  for (int cs = 0; cs < 256; cs++) {
    int below[8];
    for (int v = 0; v < 8; v++) below[v] = (cs >> v) & 1;
    int nb[12][2], deg[12];
    for (int e = 0; e < 12; e++) { deg[e] = 0; nb[e][0] = nb[e][1] = -1; }
    for (int f = 0; f < 6; f++) {
      int ce[4], cross[4], ncross = 0;
      for (int i = 0; i < 4; i++) {
        int a = face[f][i], b = face[f][(i + 1) % 4];
        ce[i] = edge_between(a, b);
        cross[i] = below[a] != below[b];
        ncross += cross[i];
      }
      int seg[2][2], nseg = 0;
      if (ncross == 2) {
        int k = 0;
        for (int i = 0; i < 4; i++) if (cross[i]) seg[0][k++] = ce[i];
        nseg = 1;
      } else if (ncross == 4) {
        for (int i = 0; i < 4; i++) {
          int c = face[f][i];
          if (below[c]) { /* corner i is between edges (i-1) and i */
            seg[nseg][0] = ce[(i + 3) % 4];
            seg[nseg][1] = ce[i];
            nseg++;
          }
        }
      }
      for (int s2 = 0; s2 < nseg; s2++) {
        int a = seg[s2][0], b = seg[s2][1];
        nb[a][deg[a]++] = b;
        nb[b][deg[b]++] = a;
      }
    }
    int used[12] = {0};
    int nt = 0;
    for (int start = 0; start < 12; start++) {
      if (used[start] || deg[start] == 0) continue;
      int loop[12], m = 0, prev = -1, cur = start;
      do {
        loop[m++] = cur;
        used[cur] = 1;
        int nx = (nb[cur][0] != prev) ? nb[cur][0] : nb[cur][1];
        prev = cur;
        cur = nx;
      } while (cur != start);
      /* orientation: Newell normal against the below->above direction */
      double P[12][3];
      double g[3] = {0, 0, 0};
      for (int i = 0; i < m; i++) {
        int lo, hi;
        edge_corners(loop[i], &lo, &hi);
        P[i][0] = 0.5 * ((lo & 1) + (hi & 1));
        P[i][1] = 0.5 * (((lo >> 1) & 1) + ((hi >> 1) & 1));
        P[i][2] = 0.5 * (((lo >> 2) & 1) + ((hi >> 2) & 1));
        int ax = loop[i] / 4;
        g[ax] += below[lo] ? 1.0 : -1.0; /* lo below -> f increases toward hi */
      }
      double N[3] = {0, 0, 0};
      for (int i = 0; i < m; i++) {
        const double *a = P[i], *b = P[(i + 1) % m];
        N[0] += (a[1] - b[1]) * (a[2] + b[2]);
        N[1] += (a[2] - b[2]) * (a[0] + b[0]);
        N[2] += (a[0] - b[0]) * (a[1] + b[1]);
      }
      if (N[0] * g[0] + N[1] * g[1] + N[2] * g[2] < 0) {
        for (int i = 1, j = m - 1; i < j; i++, j--) { int t = loop[i]; loop[i] = loop[j]; loop[j] = t; }
      }
      for (int i = 1; i + 1 < m; i++) {
        tri[cs][3 * nt] = (int8_t)loop[0];
        tri[cs][3 * nt + 1] = (int8_t)loop[i];
        tri[cs][3 * nt + 2] = (int8_t)loop[i + 1];
        nt++;
      }
    }
    ntri[cs] = (uint8_t)nt;
    for (int i = 3 * nt; i < 3 * ORC_MC_MAXTRI; i++) tri[cs][i] = -1;
  }
}

void orc_mc_cases(const float *f, const int64_t d[3], float k, uint8_t *cases) {
  int64_t cd[3] = {d[0] - 1, d[1] - 1, d[2] - 1};
  if (cd[0] <= 0 || cd[1] <= 0 || cd[2] <= 0) return;
#pragma omp parallel for schedule(static)
  for (int64_t z = 0; z < cd[0]; z++)
    for (int64_t y = 0; y < cd[1]; y++)
      for (int64_t x = 0; x < cd[2]; x++) {
        int c = 0;
        for (int v = 0; v < 8; v++) {
          int dx = v & 1, dy = (v >> 1) & 1, dz = (v >> 2) & 1;
          if (f[idx3(d, z + dz, y + dy, x + dx)] < k) c |= 1 << v;
        }
        cases[idx3(cd, z, y, x)] = (uint8_t)c;
      }
}

/* Marching cubes over a field whose point (0,0,0) sits at grid coordinates
 * org (x, y, z) of a larger field: positions use the larger field's
 * coordinates. */
static int mc_impl(const float *f, const int64_t d[3], const int64_t org[3], float k, float spacing, float *verts,
                   int64_t cap_v, int32_t *tris, int64_t cap_t, int64_t counts[2]) {
  static uint8_t ntri[256];
  static int8_t tab[256][3 * ORC_MC_MAXTRI];
  static int have = 0;
  if (!have) { orc_mc_table(ntri, tab); have = 1; }
  int64_t N = d[0] * d[1] * d[2];
  /* vertex ids: points in lexicographic order, then axis x, y, z (R13) */
  int64_t *vid = (int64_t *)malloc(sizeof(int64_t) * 3 * (size_t)N);
  if (!vid) return ORC_E_NOMEM;
  int64_t nv = 0;
  for (int64_t z = 0; z < d[0]; z++)
    for (int64_t y = 0; y < d[1]; y++)
      for (int64_t x = 0; x < d[2]; x++) {
        int64_t i = idx3(d, z, y, x);
        int64_t c[3] = {x, y, z};
        for (int a = 0; a < 3; a++) {
          vid[3 * i + a] = -1;
          int64_t n[3] = {x, y, z};
          n[a] += 1;
          int64_t lim = (a == 0) ? d[2] : (a == 1) ? d[1] : d[0];
          if (n[a] >= lim) continue;
          float fa = f[i], fb = f[idx3(d, n[2], n[1], n[0])];
          if ((fa < k) == (fb < k)) continue;
          if (nv < cap_v) {
            /* position (R11): t = (k - fa) / (fb - fa) along the edge */
            float num = k - fa, den = fb - fa;
            float t = num / den;
            for (int b = 0; b < 3; b++) {
              float pc = (float)(c[b] + org[b]);
              if (b == a) pc = pc + t;
              verts[3 * nv + b] = pc * spacing;
            }
          }
          vid[3 * i + a] = nv++;
        }
      }
  int64_t nt = 0;
  int over = nv > cap_v;
  for (int64_t z = 0; z + 1 < d[0]; z++)
    for (int64_t y = 0; y + 1 < d[1]; y++)
      for (int64_t x = 0; x + 1 < d[2]; x++) {
        int cs = 0;
        for (int v = 0; v < 8; v++) {
          int dx = v & 1, dy = (v >> 1) & 1, dz = (v >> 2) & 1;
          if (f[idx3(d, z + dz, y + dy, x + dx)] < k) cs |= 1 << v;
        }
        for (int t = 0; t < ntri[cs]; t++) {
          if (nt < cap_t) {
            for (int j = 0; j < 3; j++) {
              int e = tab[cs][3 * t + j];
              int lo, hi;
              edge_corners(e, &lo, &hi);
              int64_t px = x + (lo & 1), py = y + ((lo >> 1) & 1), pz = z + ((lo >> 2) & 1);
              tris[3 * nt + j] = (int32_t)vid[3 * idx3(d, pz, py, px) + e / 4];
            }
          }
          nt++;
        }
      }
  free(vid);
  counts[0] = nv;
  counts[1] = nt;
  if (over || nt > cap_t) return ORC_E_CAPACITY;
  return ORC_OK;
}

int orc_mc(const float *f, const int64_t d[3], float k, float spacing, float *verts,
           int64_t cap_v, int32_t *tris, int64_t cap_t, int64_t counts[2]) {
  const int64_t org[3] = {0, 0, 0};
  return mc_impl(f, d, org, k, spacing, verts, cap_v, tris, cap_t, counts);
}

/* Block merging for extraction (reading R21): the blocks whose stored range
 * can hold a crossing of an isovalue in [kmin, kmax] (min < max, min < kmax,
 * kmin <= max) merged into their bounding box of points, lo..hi per axis
 * (z, y, x); *found = 0 when there is none. */
int orc_block_box(const uint8_t *s, size_t n, float kmin, float kmax, int64_t lo[3], int64_t hi[3], int *found) {
  orc_info I;
  int rc = orc_stream_info(s, n, &I);
  if (rc) return rc;
  const size_t btab = HEADER_BYTES + 16 * (size_t)I.nblocks * (size_t)I.levels;
  *found = 0;
  for (int a = 0; a < 3; a++) { lo[a] = INT64_MAX; hi[a] = -1; }
  for (int64_t b = 0; b < I.nblocks; b++) {
    const float mn = getf(s + btab + 16 * (size_t)b), mx = getf(s + btab + 16 * (size_t)b + 4);
    if (!(mn < mx && mn < kmax && kmin <= mx)) continue;
    int64_t o[3], h[3];
    unit_extent(s, &I, b, o, h);
    for (int a = 0; a < 3; a++) {
      if (o[a] < lo[a]) lo[a] = o[a];
      if (h[a] > hi[a]) hi[a] = h[a];
    }
    *found = 1;
  }
  return ORC_OK;
}

/* Marching cubes over the box lo..hi (z, y, x; inclusive) of a field, with
 * the field's coordinates. */
int orc_mc_box(const float *f, const int64_t d[3], const int64_t lo[3], const int64_t hi[3], float k, float spacing,
               float *verts, int64_t cap_v, int32_t *tris, int64_t cap_t, int64_t counts[2]) {
  int64_t bd[3];
  for (int a = 0; a < 3; a++) {
    if (lo[a] < 0 || hi[a] >= d[a] || lo[a] > hi[a]) return ORC_E_INVAL;
    bd[a] = hi[a] - lo[a] + 1;
  }
  float *sub = (float *)malloc(sizeof(float) * (size_t)(bd[0] * bd[1] * bd[2]));
  if (!sub) return ORC_E_NOMEM;
  for (int64_t z = 0; z < bd[0]; z++)
    for (int64_t y = 0; y < bd[1]; y++)
      for (int64_t x = 0; x < bd[2]; x++) sub[idx3(bd, z, y, x)] = f[idx3(d, lo[0] + z, lo[1] + y, lo[2] + x)];
  const int64_t org[3] = {lo[2], lo[1], lo[0]};
  int rc = mc_impl(sub, bd, org, k, spacing, verts, cap_v, tris, cap_t, counts);
  free(sub);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* the paper's error translation (Sec. II.B)                                */
/* ------------------------------------------------------------------------ */

static int cmp_double(const void *a, const void *b) {
  double x = *(const double *)a, y = *(const double *)b;
  return (x > y) - (x < y);
}

double orc_topology_error_bound(const float *f, const int64_t d[3], const float *iso,
                                int n_iso, int64_t nth, int64_t *n_d) {
  /* (1) every grid edge (s0, s1) with k strictly between its end values;
   * (2) d0 = |k - s0| and d1 = |s1 - k| of every such edge into D;
   * (3) the smallest (or n-th smallest) entry of D. */
  int64_t cap = 1024, m = 0;
  double *D = (double *)malloc(sizeof(double) * (size_t)cap);
  for (int j = 0; j < n_iso; j++) {
    double k = iso[j];
    for (int64_t z = 0; z < d[0]; z++)
      for (int64_t y = 0; y < d[1]; y++)
        for (int64_t x = 0; x < d[2]; x++) {
          int64_t c[3] = {x, y, z};
          for (int a = 0; a < 3; a++) {
            int64_t n[3] = {c[0], c[1], c[2]};
            n[a]++;
            int64_t lim = (a == 0) ? d[2] : (a == 1) ? d[1] : d[0];
            if (n[a] >= lim) continue;
            double s0 = f[idx3(d, z, y, x)], s1 = f[idx3(d, n[2], n[1], n[0])];
            if (s0 > s1) { double t = s0; s0 = s1; s1 = t; }
            if (!(s0 < k && k < s1)) continue;
            if (m + 2 > cap) { cap *= 2; D = (double *)realloc(D, sizeof(double) * (size_t)cap); }
            D[m++] = k - s0;
            D[m++] = s1 - k;
          }
        }
  }
  *n_d = m;
  double r = INFINITY;
  if (m > 0) {
    qsort(D, (size_t)m, sizeof(double), cmp_double);
    int64_t i = nth < 1 ? 0 : (nth > m ? m - 1 : nth - 1);
    r = D[i];
  }
  free(D);
  return r;
}
