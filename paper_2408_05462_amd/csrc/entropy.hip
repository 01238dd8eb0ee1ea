// entropy.hip -- the entropy stage over a CHR stream on gfx950: an order-0
// canonical Huffman code over the stream's bytes, for the network leg of the
// in-transit workflow (Sec. III).  The code is textbook: Huffman lengths by
// the two-queue construction, the length limit of JPEG (ITU-T T.81, Annex
// K.3), RFC 1951's canonical codes; the byte layout is documented in
// include/chr.h.
//
// Encoding: a histogram (LDS bins per workgroup, one global add per bin), the
// code table by one workgroup (parallel ranks for the two sorts, one wave for
// the Huffman merge), per-chunk bit counts (one wave per 512-byte chunk), a
// scan of the chunks' word counts, and the packing (one wave per chunk: lane
// bit offsets by a wave scan, codes OR-ed into the chunk's words in LDS,
// then written out).  Decoding: one lane per chunk, a 4096-entry table of
// the 12-bit windows in LDS.
#include <algorithm>

#include <cstring>

#include "capi_internal.h"
#include "chr_plan.h"
#include "scan.h"

namespace chr {
namespace {

constexpr int kBS = 256;
constexpr int kWaves = kBS / kWave;
constexpr uint32_t kChunk = 512;      // bytes per chunk
constexpr int kMaxLen = 12;           // longest code
constexpr uint32_t kMagicH = 0x48524843u;
constexpr int kLenOff = 64, kOffOff = 320;
constexpr uint32_t kChunkWords = (kChunk * kMaxLen + 31) / 32;

struct EntTable {
  uint32_t hist[256];
  uint32_t rcode[256];   // codes, bit-reversed (first code bit lowest)
  uint8_t len[256];
};

struct EntPlan {
  const uint8_t *in;
  uint64_t n, nch;
  uint8_t *out;
  uint64_t cap, base;    // capacity, byte offset of the bit area
  EntTable *tab;
  uint64_t *csize, *woff;
  uint64_t *result;      // [0] encoded bytes, [1] status (0 or CHR_E_CAPACITY)
};

__host__ __device__ inline uint64_t bit_area(uint64_t nch) { return ((uint64_t)kOffOff + 4 * (nch + 1) + 7) & ~7ull; }

__global__ __launch_bounds__(kBS) void k_ent_clear(EntPlan E) {
  for (int i = threadIdx.x; i < 256; i += kBS) E.tab->hist[i] = 0u;
}

// Byte histogram: 8 bytes per load, eight loads of a thread in flight
// together, LDS bins, one global add per bin.
__global__ __launch_bounds__(kBS) void k_ent_hist(EntPlan E) {
  __shared__ uint32_t h[256];
  for (int i = threadIdx.x; i < 256; i += kBS) h[i] = 0u;
  __syncthreads();
  const uint64_t n8 = E.n / 8;
  const uint64_t *w = reinterpret_cast<const uint64_t *>(E.in);
  const uint64_t stride = (uint64_t)gridDim.x * kBS;
  for (uint64_t i = (uint64_t)blockIdx.x * kBS + threadIdx.x; i < n8; i += 8 * stride) {
    uint64_t v[8];
#pragma unroll
    for (int u = 0; u < 8; u++) {
      const uint64_t j = i + (uint64_t)u * stride;
      v[u] = j < n8 ? w[j] : 0ull;
    }
#pragma unroll
    for (int u = 0; u < 8; u++) {
      if (i + (uint64_t)u * stride >= n8) break;
#pragma unroll
      for (int b = 0; b < 8; b++) atomicAdd(&h[(v[u] >> (8 * b)) & 255u], 1u);
    }
  }
  if (blockIdx.x == 0)
    for (uint64_t i = 8 * n8 + threadIdx.x; i < E.n; i += kBS) atomicAdd(&h[E.in[i]], 1u);
  __syncthreads();
  for (int i = threadIdx.x; i < 256; i += kBS)
    if (h[i]) atomicAdd(&E.tab->hist[i], h[i]);
}

// The code table (one workgroup of 256 threads, thread s for byte value s).
// The Huffman merge runs on wave 0 in uniform control flow with both queues
// held in vector registers across the lanes (a pick reads the consumed
// queue's next entry with one readlane); the leaf depths follow by pointer
// jumping over the parent links.
__global__ __launch_bounds__(256) void k_ent_table(EntPlan E) {
  __shared__ __align__(16) uint32_t hs[256];
  __shared__ int order[256];      // present values by (count, value) increasing
  __shared__ int bits[512];       // codes per length
  __shared__ int par[512], anc[512], dep[512];
  __shared__ uint32_t lw[256];    // leaf weights in queue order, then leaves consumed per merge step
  __shared__ int blc[kMaxLen + 1];
  __shared__ uint32_t nextc[kMaxLen + 1];
  __shared__ int wl[kWaves][kMaxLen + 1];   // codes per length in each wave
  __shared__ int maxd_s, m_s;
  const int s = threadIdx.x, lane = lane_id(), wave = s / kWave;
  const uint32_t c = E.tab->hist[s];
  hs[s] = c;
  for (int i = s; i < 512; i += 256) bits[i] = 0;
  if (s <= kMaxLen) blc[s] = 0;
  if (s == 0) { maxd_s = 0; m_s = 0; }
  __syncthreads();
  {
    const unsigned long long pm = __ballot(c != 0u);
    if (lane == 0) atomicAdd(&m_s, __popcll(pm));
  }
  // ranks among the present values: rk by (count, value) increasing, r2 by
  // (count decreasing, value); both from one pass over the counts (for an
  // absent value they are not used)
  int rk = 0, r2 = 0;
  const uint4 *h4 = reinterpret_cast<const uint4 *>(hs);   // four counts per LDS read
#pragma unroll 8
  for (int t4 = 0; t4 < 64; t4++) {
    const uint4 q = h4[t4];
    const uint32_t ct[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const int t = 4 * t4 + i;
      const int e = ct[i] == c && t < s;
      rk += (int)(ct[i] - 1u < c - 1u) + e;   // 0 < count < c
      r2 += (int)(ct[i] > c) + e;
    }
  }
  __syncthreads();
  const int m = m_s;
  if (c) order[rk] = s;
  __syncthreads();
  if (s < m) lw[s] = hs[order[s]];
  __syncthreads();
  // two-queue Huffman on wave 0: leaves 0..m-1 in order, internal node j
  // (tree node m + j) made at step j; the lighter front is taken, a leaf
  // first on a tie (weights fit 32 bits: they sum to at most n < 2^32)
  const int nn = 2 * m - 1;   // tree nodes when m >= 2
  // (the wave test through readfirstlane, so the compiler sees a uniform
  // branch and keeps the merge's state in scalar registers)
  if (m >= 2 && __builtin_amdgcn_readfirstlane(s) < kWave) {
    // Wave-uniform, with both queues in vector registers: lane i holds
    // entries i, i + 64, i + 128 and i + 192.  Each queue is read through
    // the register of its front's 64 entries (switched at those boundaries),
    // so a pick reads its next front with one readlane, and a new node goes
    // into the register being filled with one lane select.  The parent links
    // are not written here: each step records how many leaves have been
    // consumed, and the links follow from that afterwards.
    const uint32_t ul = (uint32_t)lane;
    const uint32_t L1 = lw[ul + 64], L2 = lw[ul + 128], L3 = lw[ul + 192];
    uint32_t CL = lw[ul];          // leaves 64 (qi / 64) ..
    uint32_t N1 = 0, N2 = 0;       // finished nodes 64..127 and 128..191
    uint32_t CW = 0;               // nodes 64 (made / 64) .. made - 1
    uint32_t CR = 0;               // nodes 64 (qj / 64) .., once finished
    uint32_t CQ = 0;               // leaves consumed after steps 64 (step / 64) ..
    auto rl = [](uint32_t r, uint32_t i) { return (uint32_t)__builtin_amdgcn_readlane((int)r, (int)(i & 63u)); };
    const uint32_t mu = (uint32_t)__builtin_amdgcn_readfirstlane(m);
    uint32_t qi = 0, qj = 0, made = 0;
    uint32_t a = rl(CL, 0), b = 0;   // fronts: leaf qi (qi < m), node qj (qj < made)
    auto u = [](uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); };
    for (uint32_t step = 0; step + 1 < mu; step++) {
      uint32_t wsum = 0;
      for (int t = 0; t < 2; t++) {
        const uint32_t leaf = u((uint32_t)(qi < mu) & ((uint32_t)(qj >= made) | (uint32_t)(a <= b)));
        wsum += leaf ? a : b;
        qi += leaf;
        qj += leaf ^ 1u;
        if ((qi & 63u) == 0u && leaf) CL = qi == 64u ? L1 : qi == 128u ? L2 : L3;
        if ((qj & 63u) == 0u && !leaf && (qj >> 6) < (made >> 6)) CR = qj == 64u ? N1 : N2;
        a = u(rl(CL, qi));
        b = u(rl((qj >> 6) == (made >> 6) ? CW : CR, qj));
      }
      CW = ul == (made & 63u) ? wsum : CW;
      CQ = ul == (step & 63u) ? qi : CQ;
      made++;
      if ((made & 63u) == 0u) {
        // the register being filled is complete (made <= 255: at most three times)
        if (made == 128u) N1 = CW;
        else if (made == 192u) N2 = CW;
        if ((qj >> 6) == ((made - 1u) >> 6)) CR = CW;
        CW = 0;
      }
      if ((step & 63u) == 63u) lw[(step & ~63u) + ul] = CQ;
      if (qj + 1 == made) b = wsum;   // the node queue was empty: the new node is its front
    }
    lw[((mu - 2u) & ~63u) + ul] = CQ;
  }
  __syncthreads();
  if (m >= 2) {
    // Parent links from the per-step leaf counts lw[0..m-2] (non-decreasing,
    // lw[m-2] = m): leaf i went into the node of the first step j with
    // lw[j] > i, internal node k into that of the first step j whose node
    // count 2 (j + 1) - lw[j] exceeds k.
    for (int v = s; v < nn - 1; v += 256) {
      const bool isleaf = v < m;
      const int key = isleaf ? v : v - m;
      int lo = 0, hi = m - 2;   // the answer lies in [lo, hi]
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const int cnt = isleaf ? (int)lw[mid] : 2 * (mid + 1) - (int)lw[mid];
        if (cnt > key) hi = mid;
        else lo = mid + 1;
      }
      par[v] = m + lo;
    }
    __syncthreads();
    // depth = number of ancestors, by pointer jumping (depths stay below 256)
    const int root = nn - 1;
    for (int v = s; v < nn; v += 256) {
      anc[v] = v == root ? v : par[v];
      dep[v] = v == root ? 0 : 1;
    }
    __syncthreads();
    for (int it = 0; it < 9; it++) {
      int nd[2], na[2];
      for (int u = 0; u < 2; u++) {
        const int v = s + 256 * u;
        if (v < nn) {
          const int a = anc[v];
          nd[u] = dep[v] + (a == v ? 0 : dep[a]);
          na[u] = anc[a];
        }
      }
      __syncthreads();
      for (int u = 0; u < 2; u++) {
        const int v = s + 256 * u;
        if (v < nn) {
          dep[v] = nd[u];
          anc[v] = na[u];
        }
      }
      __syncthreads();
    }
    if (s < m) {
      const int d = min(dep[s], 511);
      atomicAdd(&bits[d], 1);
      atomicMax(&maxd_s, d);
    }
  }
  __syncthreads();
  if (s == 0) {
    if (m == 1) {
      bits[1] = 1;
    } else if (m >= 2) {
      // length limit (JPEG Annex K.3): move pairs of codes up, keeping the code complete
      for (int i = maxd_s; i > kMaxLen; i--) {
        while (bits[i] > 0) {
          int j = i - 2;
          while (j > 1 && bits[j] == 0) j--;   // a complete code always has one (j >= 1)
          bits[i] -= 2;
          bits[i - 1] += 1;
          bits[j + 1] += 2;
          bits[j] -= 1;
        }
      }
    }
  }
  __syncthreads();
  // lengths to the values from the most frequent (rank r2)
  int L = 0;
  if (c) {
    int acc = 0, l = 1;
    for (; l <= kMaxLen; l++) {
      if (r2 < acc + bits[l]) break;
      acc += bits[l];
    }
    L = l;
    atomicAdd(&blc[l], 1);
  }
  // canonical codes: shorter first, consecutive in value order within a
  // length; the values of this length below s, counted by ballots per wave
  int before = 0;
  for (int l = 1; l <= kMaxLen; l++) {
    const unsigned long long mk = __ballot(L == l);
    if (lane == 0) wl[wave][l] = __popcll(mk);
    if (L == l) before = __popcll(mk & ((1ull << lane) - 1ull));
  }
  __syncthreads();
  if (s == 0) {
    uint32_t code = 0;
    for (int l = 1; l <= kMaxLen; l++) {
      code = (code + (uint32_t)(l > 1 ? blc[l - 1] : 0)) << 1;
      nextc[l] = code;
    }
  }
  __syncthreads();
  uint32_t code = 0;
  if (L) {
    for (int w = 0; w < wave; w++) before += wl[w][L];
    code = nextc[L] + (uint32_t)before;
  }
  uint32_t r = 0;
  for (int b = 0; b < L; b++) r |= ((code >> b) & 1u) << (L - 1 - b);
  E.tab->rcode[s] = r;
  E.tab->len[s] = (uint8_t)L;
}

// The 8 input bytes at b (8-aligned): one load inside the input, bytes up
// to its end otherwise (zero past it).
__device__ inline uint64_t load8(const EntPlan &E, uint64_t b) {
  if (b + 8 <= E.n) return *reinterpret_cast<const uint64_t *>(E.in + b);
  uint64_t v = 0;
  for (uint64_t i = b; i < E.n; i++) v |= (uint64_t)E.in[i] << (8 * (i - b));
  return v;
}

// Bits of each chunk (one wave per chunk, 8 bytes per lane), as 32-bit words.
__global__ __launch_bounds__(kBS) void k_ent_sizes(EntPlan E) {
  __shared__ uint8_t ln[256];
  for (int i = threadIdx.x; i < 256; i += kBS) ln[i] = E.tab->len[i];
  __syncthreads();
  const uint64_t c = (uint64_t)blockIdx.x * kWaves + wave_index();
  if (c >= E.nch) return;
  const int lane = lane_id();
  const uint64_t b0 = c * kChunk + 8 * (uint64_t)lane;
  const uint64_t v = load8(E, b0);
  uint32_t bits = 0;
#pragma unroll
  for (int b = 0; b < 8; b++)
    if (b0 + b < E.n) bits += ln[(v >> (8 * b)) & 255u];
  bits = wave_sum_dpp(bits);
  if (lane == 0) E.csize[c] = (bits + 31) / 32;
}

// The header, the code lengths and the last chunk offset; the result.
__global__ __launch_bounds__(kBS) void k_ent_header(EntPlan E) {
  const uint64_t total = E.base + 4 * E.woff[E.nch];
  const bool fits = total <= E.cap;
  if (threadIdx.x == 0) {
    E.result[0] = total;
    E.result[1] = fits ? 0ull : (uint64_t)(int64_t)CHR_E_CAPACITY;
  }
  if (!fits) return;
  uint32_t *o32 = reinterpret_cast<uint32_t *>(E.out);
  for (uint32_t i = threadIdx.x; i < 16; i += kBS) {
    uint32_t v = 0;
    if (i == 0) v = kMagicH;
    if (i == 1) v = 1u;
    if (i == 2) v = (uint32_t)E.n;
    if (i == 3) v = (uint32_t)(E.n >> 32);
    if (i == 4) v = kChunk;
    if (i == 5) v = (uint32_t)E.nch;
    if (i == 6) v = (uint32_t)total;
    if (i == 7) v = (uint32_t)(total >> 32);
    if (i == 8) v = (uint32_t)kMaxLen;
    o32[i] = v;
  }
  for (uint32_t i = threadIdx.x; i < 256; i += kBS) E.out[kLenOff + i] = E.tab->len[i];
  if (threadIdx.x == 0) {
    o32[kOffOff / 4 + E.nch] = (uint32_t)E.woff[E.nch];
    if (kOffOff + 4 * (E.nch + 1) < E.base) o32[kOffOff / 4 + E.nch + 1] = 0u;  // padding word
  }
}

// Packs chunk c (one wave): lane bit offsets by a wave scan, codes OR-ed
// into the chunk's words in LDS, the words written out with the chunk's
// offset entry.
__global__ __launch_bounds__(kBS) void k_ent_write(EntPlan E) {
  __shared__ uint32_t rcode[256];
  __shared__ uint8_t ln[256];
  __shared__ uint32_t words[kWaves][kChunkWords];
  for (int i = threadIdx.x; i < 256; i += kBS) {
    rcode[i] = E.tab->rcode[i];
    ln[i] = E.tab->len[i];
  }
  __syncthreads();
  const uint64_t total = E.base + 4 * E.woff[E.nch];
  if (total > E.cap) return;
  const uint32_t wave = wave_index();
  const uint64_t c = (uint64_t)blockIdx.x * kWaves + wave;
  if (c >= E.nch) return;
  const int lane = lane_id();
  uint32_t *wd = words[wave];
  for (uint32_t i = (uint32_t)lane; i < kChunkWords; i += kWave) wd[i] = 0u;
  const uint64_t b0 = c * kChunk + 8 * (uint64_t)lane;
  const uint64_t v8 = load8(E, b0);
  uint32_t sym[8];
  uint32_t bits = 0;
#pragma unroll
  for (int b = 0; b < 8; b++) {
    sym[b] = b0 + b < E.n ? (uint32_t)((v8 >> (8 * b)) & 255u) : 256u;
    bits += sym[b] < 256u ? ln[sym[b]] : 0u;
  }
  uint32_t pos = wave_excl_sum(bits);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int b = 0; b < 8; b++) {
    if (sym[b] < 256u) {
      const uint32_t L = ln[sym[b]], r = rcode[sym[b]];
      const uint32_t wi = pos >> 5, off = pos & 31u;
      atomicOr(&wd[wi], r << off);
      if (off + L > 32u) atomicOr(&wd[wi + 1], r >> (32u - off));
      pos += L;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
  const uint64_t w0 = E.woff[c], nwd = E.woff[c + 1] - w0;
  uint32_t *dst = reinterpret_cast<uint32_t *>(E.out + E.base) + w0;
  for (uint32_t i = (uint32_t)lane; i < nwd; i += kWave) dst[i] = wd[i];
  if (lane == 0) reinterpret_cast<uint32_t *>(E.out + kOffOff)[c] = (uint32_t)w0;
}

__global__ void k_ent_status0(int32_t *status) {
  if (threadIdx.x == 0) *status = 0;
}

// Decoding: one lane per chunk; the 12-bit windows' (value, length) in LDS.
struct DecE {
  const uint8_t *in;
  uint64_t nbytes, n, nch, base;
  uint8_t *out;
  int32_t *status;
};

__global__ __launch_bounds__(kBS) void k_ent_decode(DecE D) {
  __shared__ uint16_t tab[1 << kMaxLen];
  __shared__ int blc[kMaxLen + 1], start[kMaxLen + 1];
  __shared__ uint32_t nextc[kMaxLen + 1];
  __shared__ int wl[kWaves][kMaxLen + 1];   // codes per length in each wave
  __shared__ uint8_t sorted[256];           // the values by (length, value)
  // Canonical codes of the stored lengths (as the encoder): the codes of
  // length l are blc[l] consecutive integers from nextc[l], taken by the
  // values of that length in increasing order.  A length above the limit is
  // never written by the encoder: the stream is corrupt.
  const int s = threadIdx.x, lane = lane_id(), wave = s / kWave;
  const int L = D.in[kLenOff + s];
  const bool has = L >= 1 && L <= kMaxLen;
  if (L > kMaxLen) *D.status = CHR_E_CORRUPT;
  if (s <= kMaxLen) blc[s] = 0;
  __syncthreads();
  if (has) atomicAdd(&blc[L], 1);
  // the values of this length below s: ballots per wave, then the waves before
  int before = 0;
  for (int l = 1; l <= kMaxLen; l++) {
    const unsigned long long mk = __ballot(has && L == l);
    if (lane == 0) wl[wave][l] = __popcll(mk);
    if (has && L == l) before = __popcll(mk & ((1ull << lane) - 1ull));
  }
  __syncthreads();
  if (s == 0) {
    uint32_t code = 0;
    int acc = 0;
    for (int l = 1; l <= kMaxLen; l++) {
      code = (code + (uint32_t)(l > 1 ? blc[l - 1] : 0)) << 1;
      nextc[l] = code;
      start[l] = acc;
      acc += blc[l];
    }
  }
  __syncthreads();
  if (has) {
    for (int w = 0; w < wave; w++) before += wl[w][L];
    sorted[start[L] + before] = (uint8_t)s;
  }
  __syncthreads();
  // The window table, 16 entries per thread: window i (code bits from its
  // lowest bit) decodes as the canonical decoder reading bit by bit would,
  // the shortest length whose prefix is a code of that length; no code: 0.
  {
    uint32_t nx[kMaxLen + 1], bc[kMaxLen + 1], st[kMaxLen + 1];
#pragma unroll
    for (int l = 1; l <= kMaxLen; l++) {
      nx[l] = nextc[l];
      bc[l] = (uint32_t)blc[l];
      st[l] = (uint32_t)start[l];
    }
    for (int i = s; i < (1 << kMaxLen); i += kBS) {
      const uint32_t rev = __brev((uint32_t)i) >> (32 - kMaxLen);   // first code bit highest
      uint32_t e = 0;
      bool found = false;
#pragma unroll
      for (int l = 1; l <= kMaxLen; l++) {
        const uint32_t d = (rev >> (kMaxLen - l)) - nx[l];
        if (!found && d < bc[l]) {
          found = true;
          e = (uint32_t)sorted[st[l] + d] | ((uint32_t)l << 8);
        }
      }
      tab[i] = (uint16_t)e;
    }
  }
  __syncthreads();
  const uint64_t c = (uint64_t)blockIdx.x * kBS + threadIdx.x;
  if (c >= D.nch) return;
  const uint32_t *offs = reinterpret_cast<const uint32_t *>(D.in + kOffOff);
  const uint64_t w0 = offs[c], w1 = offs[c + 1];
  const uint64_t words = (D.nbytes - D.base) / 4;
  if (w0 >= w1 || w1 > words) {   // every chunk holds at least one code, so at least one word
    *D.status = CHR_E_CORRUPT;
    return;
  }
  const uint32_t *src = reinterpret_cast<const uint32_t *>(D.in + D.base);
  const uint64_t first = c * kChunk;
  const uint32_t len = (uint32_t)min<uint64_t>(kChunk, D.n - first);
  // A fixed schedule: every 4 symbols, the 64 bits at the current position
  // from three whole words (unconditional loads, clamped to the bit area),
  // which hold 4 codes of at most 12 bits.  Loads on a per-lane condition
  // would make the compiler wait for every outstanding load at each refill.
  // 64 decoded bytes are held in registers and written together, so stores
  // do not sit between a window's loads and their use either.
  const uint64_t wlast = words - 1;   // words >= w1 > w0 here
  uint64_t pos = 0;                   // bits consumed
  uint32_t used = 0;
  bool bad = false;
  for (uint32_t i0 = 0; i0 < len; i0 += 64) {
    uint64_t o[8];
#pragma unroll
    for (int g = 0; g < 16; g++) {
      const uint64_t wi = w0 + (pos >> 5);
      const uint32_t sh = (uint32_t)(pos & 31u);
      uint32_t a = src[min(wi, wlast)], b = src[min(wi + 1, wlast)], d = src[min(wi + 2, wlast)];
      a = wi < w1 ? a : 0u;
      b = wi + 1 < w1 ? b : 0u;
      d = wi + 2 < w1 ? d : 0u;
      uint64_t win = ((((uint64_t)b << 32) | a) >> sh) | (sh ? (uint64_t)d << (64 - sh) : 0ull);
      uint64_t acc = 0;
#pragma unroll
      for (int k = 0; k < 4; k++) {
        const bool live = i0 + (uint32_t)(4 * g + k) < len;
        const uint32_t e = tab[win & ((1u << kMaxLen) - 1u)];
        uint32_t Ls = e >> 8;
        bad |= live && Ls == 0;
        Ls = live ? (Ls ? Ls : 1u) : 0u;
        win >>= Ls;
        pos += Ls;
        acc |= (uint64_t)(e & 255u) << (8 * k);
      }
      if (g & 1) o[g >> 1] |= acc << 32;
      else o[g >> 1] = acc;
    }
    uint8_t *dst = D.out + first + i0;
    if (i0 + 64 <= len) {
#pragma unroll
      for (int g = 0; g < 8; g++) reinterpret_cast<uint64_t *>(dst)[g] = o[g];
    } else {
      for (uint32_t k = 0; i0 + k < len; k++) dst[k] = (uint8_t)(o[k >> 3] >> (8 * (k & 7u)));
    }
  }
  used = pos > 0xffffffffull ? 0xffffffffu : (uint32_t)pos;
  bad |= (uint64_t)used > (w1 - w0) * 32;  // read past the chunk's bits
  if (bad) *D.status = CHR_E_CORRUPT;
}

}  // namespace

uint64_t entropy_bound(uint64_t n) {
  const uint64_t nch = (n + kChunk - 1) / kChunk;
  return bit_area(nch) + 4 * ((n * (uint64_t)kMaxLen + 31) / 32 + nch);
}

size_t entropy_workspace(uint64_t n) {
  const uint64_t nch = (n + kChunk - 1) / kChunk;
  size_t o = (sizeof(EntTable) + 255) & ~(size_t)255;
  o += (8 * nch + 255) & ~(size_t)255;                              // chunk word counts
  o += (8 * (nch + 1) + 255) & ~(size_t)255;                        // offsets
  o += (8 * (size_t)scan_tmp_elems((int64_t)nch) + 255) & ~(size_t)255;  // scan scratch
  return o;
}

int launch_entropy_encode(const uint8_t *in, uint64_t n, uint8_t *out, uint64_t cap, uint64_t *result, void *ws,
                          hipStream_t s) {
  EntPlan E;
  E.in = in;
  E.n = n;
  E.nch = (n + kChunk - 1) / kChunk;
  E.out = out;
  E.cap = cap;
  E.base = bit_area(E.nch);
  uint8_t *w = static_cast<uint8_t *>(ws);
  size_t o = 0;
  E.tab = reinterpret_cast<EntTable *>(w + o);
  o += (sizeof(EntTable) + 255) & ~(size_t)255;
  E.csize = reinterpret_cast<uint64_t *>(w + o);
  o += (8 * E.nch + 255) & ~(size_t)255;
  E.woff = reinterpret_cast<uint64_t *>(w + o);
  o += (8 * (E.nch + 1) + 255) & ~(size_t)255;
  uint64_t *tmp = reinterpret_cast<uint64_t *>(w + o);
  E.result = result;
  k_ent_clear<<<1, kBS, 0, s>>>(E);
  const uint64_t g = std::min<uint64_t>(std::max<uint64_t>((n / 8 + kBS - 1) / kBS, 1), 512);
  k_ent_hist<<<dim3((unsigned)g), dim3(kBS), 0, s>>>(E);
  k_ent_table<<<1, 256, 0, s>>>(E);
  const unsigned gw = (unsigned)std::max<uint64_t>((E.nch + kWaves - 1) / kWaves, 1);
  if (E.nch) k_ent_sizes<<<dim3(gw), dim3(kBS), 0, s>>>(E);
  scan_u64(E.csize, E.woff, (int64_t)E.nch, tmp, s);
  k_ent_header<<<1, kBS, 0, s>>>(E);
  if (E.nch) k_ent_write<<<dim3(gw), dim3(kBS), 0, s>>>(E);
  return 0;
}

int launch_entropy_decode(const uint8_t *in, uint64_t nbytes, uint64_t n, uint64_t nch, uint8_t *out, int32_t *status,
                          hipStream_t s) {
  DecE D;
  D.in = in;
  D.nbytes = nbytes;
  D.n = n;
  D.nch = nch;
  D.base = bit_area(nch);
  D.out = out;
  D.status = status;
  if (nch) k_ent_decode<<<dim3((unsigned)((nch + kBS - 1) / kBS)), dim3(kBS), 0, s>>>(D);
  return 0;
}

uint64_t entropy_bit_area(uint64_t nch) { return bit_area(nch); }
uint32_t entropy_chunk() { return kChunk; }

}  // namespace chr

// ---- C ABI -------------------------------------------------------------------

using namespace chr;

namespace {
bool aligned8(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }
uint32_t hget32(const uint8_t *p) { uint32_t v; std::memcpy(&v, p, 4); return v; }
uint64_t hget64(const uint8_t *p) { uint64_t v; std::memcpy(&v, p, 8); return v; }
}  // namespace

extern "C" {

size_t chr_entropy_bound(uint64_t n) { return (size_t)entropy_bound(n); }

size_t chr_entropy_workspace(uint64_t n) { return entropy_workspace(n); }

int chr_entropy_encode(const void *d_in, uint64_t n, void *d_out, size_t capacity, uint64_t *d_result, void *d_ws,
                       size_t ws_bytes, void *stream) {
  if ((!d_in && n) || !d_out || !d_result || !d_ws) return api_fail(CHR_E_INVAL, "NULL device pointer");
  if (!aligned8(d_in) || !aligned8(d_out) || !aligned8(d_result))
    return api_fail(CHR_E_INVAL, "buffers must be 8-byte aligned");
  if (n >= (1ull << 32)) return api_fail(CHR_E_INVAL, "entropy stage: n must be below 2^32");
  const size_t need = entropy_workspace(n);
  if (ws_bytes < need) return api_fail(CHR_E_NOMEM, "workspace too small: need " + std::to_string(need));
  launch_entropy_encode(static_cast<const uint8_t *>(d_in), n, static_cast<uint8_t *>(d_out), capacity, d_result,
                        d_ws, static_cast<hipStream_t>(stream));
  return api_check_launch("chr_entropy_encode");
}

int chr_entropy_info(const void *h_head, size_t head_bytes, uint64_t *n, uint64_t *total) {
  if (!h_head || !n || !total) return api_fail(CHR_E_INVAL, "NULL argument");
  const uint8_t *h = static_cast<const uint8_t *>(h_head);
  if (head_bytes < 64 || hget32(h) != 0x48524843u || hget32(h + 4) != 1u)
    return api_fail(CHR_E_CORRUPT, "not an entropy-stage stream (magic/version)");
  const uint64_t nn = hget64(h + 8);
  if (hget32(h + 16) != entropy_chunk() || hget32(h + 32) != 12u ||
      (uint64_t)hget32(h + 20) != (nn + entropy_chunk() - 1) / entropy_chunk())
    return api_fail(CHR_E_CORRUPT, "entropy stream: unsupported chunk size or code length, or inconsistent header");
  *n = nn;
  *total = hget64(h + 24);
  return CHR_OK;
}

int chr_entropy_decode(const void *h_head, const void *d_in, uint64_t nbytes, void *d_out, uint64_t out_capacity,
                       int32_t *d_status, void *stream) {
  uint64_t n = 0, total = 0;
  int rc = chr_entropy_info(h_head, 64, &n, &total);
  if (rc) return rc;
  if (!d_in || (!d_out && n) || !d_status) return api_fail(CHR_E_INVAL, "NULL device pointer");
  if (!aligned8(d_in) || !aligned8(d_out)) return api_fail(CHR_E_INVAL, "buffers must be 8-byte aligned");
  const uint64_t nch = (n + entropy_chunk() - 1) / entropy_chunk();
  if (total != nbytes || nbytes < entropy_bit_area(nch))
    return api_fail(CHR_E_CORRUPT, "entropy stream: size does not match its header");
  if (out_capacity < n) return api_fail(CHR_E_CAPACITY, "output below the decoded size " + std::to_string(n));
  hipStream_t s = static_cast<hipStream_t>(stream);
  k_ent_status0<<<1, 64, 0, s>>>(d_status);
  launch_entropy_decode(static_cast<const uint8_t *>(d_in), nbytes, n, nch, static_cast<uint8_t *>(d_out), d_status,
                        s);
  return api_check_launch("chr_entropy_decode");
}

}  // extern "C"
