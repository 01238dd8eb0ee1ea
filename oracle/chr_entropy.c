/*
 * chr_entropy.c -- CPU oracle of the entropy stage over a CHR stream.
 *
 * TEST INFRASTRUCTURE ONLY, like chr_oracle.c: the reference the GPU entropy
 * stage is checked against.  It shares no code with the GPU library.
 *
 * The paper sends the compressed stream over the network (Sec. III, the
 * in-transit workflow) and leaves the coding of the stream's bytes open.
 * This stage is an order-0 Huffman code over the stream's bytes, restated
 * from the textbook algorithms it uses:
 *   - code lengths: Huffman's construction, taking the two lightest of the
 *     sorted leaves and the internal nodes in creation order (two queues);
 *   - length limit: the adjustment of the per-length code counts of the JPEG
 *     standard (ITU-T T.81, Annex K.3), which moves pairs of codes upward
 *     while keeping the code complete;
 *   - codes: the canonical assignment of RFC 1951 Sec. 3.2.2 (codes of one
 *     length consecutive in symbol order, shorter codes first);
 *   - bits: LSB-first within little-endian 32-bit words, each code written
 *     most-significant bit first (so the decoder reads bit-reversed codes).
 *
 * Format (little-endian):
 *   0 u32 magic "CHRH"  4 u32 version 1  8 u64 n (decoded bytes)
 *   16 u32 chunk bytes  20 u32 nchunks = ceil(n / chunk)  24 u64 total bytes
 *   32 u32 maximum code length  36..63 zero
 *   64 u8 code length of each byte value (0: absent)
 *   320 u32 word offset of each chunk's bits, nchunks + 1 entries (the last
 *       one is the bit area's length in words), then zero padding to 8 bytes
 *   bit area: chunk c codes bytes [c*chunk, min((c+1)*chunk, n)), from word
 *       offset[c], its last word zero-padded.
 * One byte value alone gets a 1-bit code; an empty input has no chunks.
 */
#include "chr_oracle.h"

#include <stdlib.h>
#include <string.h>

#define ENT_MAGIC 0x48524843u /* "CHRH" */
#define ENT_VERSION 1u
#define ENT_LEN_OFF 64
#define ENT_OFF_OFF 320

static void e_put32(uint8_t *p, uint32_t v) { for (int i = 0; i < 4; i++) p[i] = (uint8_t)(v >> (8 * i)); }
static void e_put64(uint8_t *p, uint64_t v) { for (int i = 0; i < 8; i++) p[i] = (uint8_t)(v >> (8 * i)); }
static uint32_t e_get32(const uint8_t *p) { uint32_t v = 0; for (int i = 0; i < 4; i++) v |= (uint32_t)p[i] << (8 * i); return v; }
static uint64_t e_get64(const uint8_t *p) { uint64_t v = 0; for (int i = 0; i < 8; i++) v |= (uint64_t)p[i] << (8 * i); return v; }

/* symbols in increasing (count, value) order */
static uint64_t *g_hist;
static int by_count_up(const void *a, const void *b) {
  const int x = *(const int *)a, y = *(const int *)b;
  if (g_hist[x] != g_hist[y]) return g_hist[x] < g_hist[y] ? -1 : 1;
  return x - y;
}
/* symbols in decreasing count, increasing value order */
static int by_count_down(const void *a, const void *b) {
  const int x = *(const int *)a, y = *(const int *)b;
  if (g_hist[x] != g_hist[y]) return g_hist[x] > g_hist[y] ? -1 : 1;
  return x - y;
}

int orc_huff_lengths(const uint64_t hist[256], int maxlen, uint8_t len[256]) {
  if (maxlen < 8 || maxlen > 31) return ORC_E_INVAL;
  int sym[256], m = 0;
  for (int s = 0; s < 256; s++) {
    len[s] = 0;
    if (hist[s]) sym[m++] = s;
  }
  if (m == 0) return ORC_OK;
  if (m == 1) { len[sym[0]] = 1; return ORC_OK; }
  uint64_t hcopy[256];
  memcpy(hcopy, hist, sizeof(hcopy));
  g_hist = hcopy;
  qsort(sym, (size_t)m, sizeof(int), by_count_up);
  /* Huffman: nodes 0..m-1 are the sorted leaves, m.. the internal nodes in
   * creation order; each step joins the two lightest fronts of the two
   * queues, a leaf first when weights tie. */
  uint64_t wt[511];
  int parent[511];
  for (int i = 0; i < m; i++) wt[i] = hist[sym[i]];
  int qi = 0, qj = m, made = m;
  for (int step = 0; step < m - 1; step++) {
    int pick[2];
    for (int t = 0; t < 2; t++) {
      if (qi < m && (qj >= made || wt[qi] <= wt[qj])) pick[t] = qi++;
      else pick[t] = qj++;
    }
    wt[made] = wt[pick[0]] + wt[pick[1]];
    parent[pick[0]] = parent[pick[1]] = made;
    made++;
  }
  int depth[511];
  depth[made - 1] = 0;
  for (int v = made - 2; v >= 0; v--) depth[v] = depth[parent[v]] + 1;
  /* codes per length, then the length limit (JPEG Annex K.3) */
  int bits[512] = {0};
  int maxd = 0;
  for (int i = 0; i < m; i++) {
    bits[depth[i]]++;
    if (depth[i] > maxd) maxd = depth[i];
  }
  for (int i = maxd; i > maxlen; i--) {
    while (bits[i] > 0) {
      int j = i - 2;
      while (bits[j] == 0) j--;
      bits[i] -= 2;
      bits[i - 1] += 1;
      bits[j + 1] += 2;
      bits[j] -= 1;
    }
  }
  /* the lengths go to the symbols from the most frequent */
  qsort(sym, (size_t)m, sizeof(int), by_count_down);
  int k = 0;
  for (int l = 1; l <= maxlen; l++)
    for (int c = 0; c < bits[l]; c++) len[sym[k++]] = (uint8_t)l;
  return ORC_OK;
}

int orc_huff_codes(const uint8_t len[256], uint32_t code[256]) {
  int count[32] = {0};
  for (int s = 0; s < 256; s++) {
    if (len[s] > 31) return ORC_E_INVAL;
    count[len[s]]++;
  }
  count[0] = 0;
  uint32_t next[32];
  uint32_t c = 0;
  for (int l = 1; l < 32; l++) {
    c = (c + (uint32_t)count[l - 1]) << 1;
    next[l] = c;
  }
  for (int s = 0; s < 256; s++) code[s] = len[s] ? next[len[s]]++ : 0u;
  return ORC_OK;
}

static uint32_t reverse_bits(uint32_t v, int n) {
  uint32_t r = 0;
  for (int i = 0; i < n; i++) r |= ((v >> i) & 1u) << (n - 1 - i);
  return r;
}

static uint64_t bitarea_off(uint64_t nchunks) {
  const uint64_t o = ENT_OFF_OFF + 4 * (nchunks + 1);
  return (o + 7) & ~(uint64_t)7;
}

uint64_t orc_entropy_bound(uint64_t n, uint32_t chunk, int maxlen) {
  if (chunk == 0) return 0;
  const uint64_t nch = (n + chunk - 1) / chunk;
  return bitarea_off(nch) + 4 * ((n * (uint64_t)maxlen + 31) / 32 + nch);
}

int orc_entropy_encode(const uint8_t *in, uint64_t n, uint32_t chunk, int maxlen, uint8_t *out, uint64_t cap,
                       uint64_t *out_bytes) {
  if (chunk == 0 || (chunk & 3) || maxlen < 8 || maxlen > 24) return ORC_E_INVAL;
  const uint64_t nch = (n + chunk - 1) / chunk;
  if (nch >= 0xffffffffull) return ORC_E_INVAL;
  uint64_t hist[256] = {0};
  for (uint64_t i = 0; i < n; i++) hist[in[i]]++;
  uint8_t len[256];
  uint32_t code[256];
  int rc = orc_huff_lengths(hist, maxlen, len);
  if (rc) return rc;
  orc_huff_codes(len, code);
  /* word offsets of the chunks */
  uint64_t *woff = (uint64_t *)malloc(sizeof(uint64_t) * (nch + 1));
  if (!woff) return ORC_E_NOMEM;
  woff[0] = 0;
  for (uint64_t c = 0; c < nch; c++) {
    uint64_t bits = 0;
    const uint64_t e = (c + 1) * chunk < n ? (c + 1) * chunk : n;
    for (uint64_t i = c * chunk; i < e; i++) bits += len[in[i]];
    woff[c + 1] = woff[c] + (bits + 31) / 32;
  }
  const uint64_t base = bitarea_off(nch), total = base + 4 * woff[nch];
  *out_bytes = total;
  if (total > cap || woff[nch] > 0xffffffffull) { free(woff); return ORC_E_CAPACITY; }
  memset(out, 0, (size_t)total);
  e_put32(out, ENT_MAGIC);
  e_put32(out + 4, ENT_VERSION);
  e_put64(out + 8, n);
  e_put32(out + 16, chunk);
  e_put32(out + 20, (uint32_t)nch);
  e_put64(out + 24, total);
  e_put32(out + 32, (uint32_t)maxlen);
  memcpy(out + ENT_LEN_OFF, len, 256);
  for (uint64_t c = 0; c <= nch; c++) e_put32(out + ENT_OFF_OFF + 4 * c, (uint32_t)woff[c]);
  for (uint64_t c = 0; c < nch; c++) {
    uint64_t bit = 32 * woff[c];
    const uint64_t e = (c + 1) * chunk < n ? (c + 1) * chunk : n;
    for (uint64_t i = c * chunk; i < e; i++) {
      const int l = len[in[i]];
      const uint32_t r = reverse_bits(code[in[i]], l);
      for (int b = 0; b < l; b++, bit++)
        if ((r >> b) & 1u) out[base + bit / 8] |= (uint8_t)(1u << (bit % 8));
    }
  }
  free(woff);
  return ORC_OK;
}

int orc_entropy_info(const uint8_t *in, uint64_t nbytes, uint64_t *n, uint32_t *chunk) {
  if (nbytes < ENT_OFF_OFF + 4 || e_get32(in) != ENT_MAGIC || e_get32(in + 4) != ENT_VERSION) return ORC_E_CORRUPT;
  *n = e_get64(in + 8);
  *chunk = e_get32(in + 16);
  return ORC_OK;
}

int orc_entropy_decode(const uint8_t *in, uint64_t nbytes, uint8_t *out, uint64_t out_cap, uint64_t *n_out) {
  uint64_t n;
  uint32_t chunk;
  if (orc_entropy_info(in, nbytes, &n, &chunk)) return ORC_E_CORRUPT;
  const uint32_t nch = e_get32(in + 20);
  const int maxlen = (int)e_get32(in + 32);
  if (chunk == 0 || (uint64_t)nch != (n + chunk - 1) / chunk || maxlen < 1 || maxlen > 24) return ORC_E_CORRUPT;
  const uint64_t base = bitarea_off(nch);
  if (base > nbytes || e_get64(in + 24) != nbytes) return ORC_E_CORRUPT;
  *n_out = n;
  if (n > out_cap) return ORC_E_CAPACITY;
  const uint8_t *len = in + ENT_LEN_OFF;
  for (int s = 0; s < 256; s++)
    if (len[s] > maxlen) return ORC_E_CORRUPT;
  /* canonical decoding: the codes of length l are the count[l] consecutive
   * values from first[l], belonging to the symbols of that length in
   * increasing order (sorted[start[l] ..]) */
  int count[25] = {0}, start[25], sorted[256], ns = 0;
  uint32_t first[25];
  for (int s = 0; s < 256; s++) count[len[s]]++;
  count[0] = 0;
  for (int l = 1, acc = 0; l <= maxlen; l++) { start[l] = acc; acc += count[l]; }
  for (int l = 1; l <= maxlen; l++)
    for (int s = 0; s < 256; s++)
      if (len[s] == l) sorted[ns++] = s;
  {
    uint32_t c = 0;
    for (int l = 1; l <= maxlen; l++) {
      c = (c + (uint32_t)count[l - 1]) << 1;
      first[l] = c;
    }
  }
  const uint64_t words = (nbytes - base) / 4;
  for (uint32_t c = 0; c < nch; c++) {
    const uint64_t w0 = e_get32(in + ENT_OFF_OFF + 4 * (uint64_t)c), w1 = e_get32(in + ENT_OFF_OFF + 4 * (uint64_t)c + 4);
    if (w0 > w1 || w1 > words) return ORC_E_CORRUPT;
    uint64_t bit = 32 * w0;
    const uint64_t bend = 32 * w1;
    const uint64_t e = ((uint64_t)c + 1) * chunk < n ? ((uint64_t)c + 1) * chunk : n;
    for (uint64_t i = (uint64_t)c * chunk; i < e; i++) {
      /* one bit at a time, most significant first */
      uint32_t v = 0;
      int found = -1;
      for (int l = 1; l <= maxlen && found < 0; l++) {
        if (bit >= bend) return ORC_E_CORRUPT;
        v = (v << 1) | ((in[base + bit / 8] >> (bit % 8)) & 1u);
        bit++;
        if (v - first[l] < (uint32_t)count[l]) found = sorted[start[l] + (int)(v - first[l])];
      }
      if (found < 0) return ORC_E_CORRUPT;
      out[i] = (uint8_t)found;
    }
  }
  return ORC_OK;
}
