// tiers.hip -- multi-tier progressive accuracy on gfx950 (Sec. II: the
// visualization side requests data at the accuracy it needs).  Tier 0 is the
// topology-preserving CHR stream of the field at the loosest bound; tier t
// is the CHR stream, without isovalues, of the binary32 residual against the
// previous tiers' reconstruction, plus an exact list of the points that
// would miss the tier's bound or change side of a candidate isovalue.  The
// container layout is documented in include/chr.h.
//
// Compression runs the single-field encoder and decoder per tier on the
// caller's stream; the container offsets are kept on the device (a running
// cursor in the workspace), so nothing waits for the host.
#include <cstring>
#include <string>

#include "capi_internal.h"
#include "chr_plan.h"
#include "scan.h"

namespace chr {
namespace {

constexpr int kBS = 256;
constexpr int kTHead = 128, kTRec = 64, kTData = kTHead + kTRec * CHR_MAX_TIERS;
constexpr uint32_t kTMagic = 0x54524843u;  // "CHRT"

__host__ __device__ inline uint64_t tpad8(uint64_t v) { return (v + 7) & ~7ull; }

// Device state of one compression (in the workspace).
struct TierState {
  uint64_t cursor;          // next free byte of the container
  int64_t status;           // first failure: CHR_E_INVAL (non-finite input), CHR_E_CAPACITY, CHR_E_CORRUPT
  uint64_t so, sb, nc, io, vo;  // the current tier's stream offset and size, corrections, list offsets
  uint64_t rec[CHR_MAX_TIERS][8];
};

struct TierIso {
  int K;
  float v[16];
};

struct TierHead {
  int T, K, levels, block, qmax;
  int64_t dims[3];
  float iso[16];
};

__global__ void k_tier_init(TierState *S) {
  uint64_t *w = reinterpret_cast<uint64_t *>(S);
  for (uint32_t i = threadIdx.x; i < sizeof(TierState) / 8; i += blockDim.x) w[i] = 0;
  __syncthreads();
  if (threadIdx.x == 0) S->cursor = kTData;
}

__global__ __launch_bounds__(kBS) void k_tier_residual(const float *__restrict__ x, const float *__restrict__ y,
                                                        float *__restrict__ r, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * kBS + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kBS)
    r[i] = __fsub_rn(x[i], y[i]);
}

__device__ inline int tier_rank(const TierIso &iso, float v) {
  int r = 0;
  for (int j = 0; j < 16; j++)
    if (j < iso.K) r += iso.v[j] <= v ? 1 : 0;
  return r;
}

// y + r' per point; a point missing the bound or changing side of a
// candidate takes x.  One wave per 64-point word: its mask and count.
__global__ __launch_bounds__(kBS) void k_tier_combine(const float *__restrict__ x, float *__restrict__ y,
                                                       const float *__restrict__ rr, uint64_t n, double e, TierIso iso,
                                                       unsigned long long *__restrict__ mask, uint64_t *__restrict__ cnt) {
  const uint64_t nw = (n + 63) / 64, stride = (uint64_t)gridDim.x * kBS;
  // whole waves step together, so each 64-point word stays in one wave
  for (uint64_t i = (uint64_t)blockIdx.x * kBS + threadIdx.x; i < 64 * nw; i += stride) {
    bool bad = false;
    if (i < n) {
      const float xv = x[i];
      const float v = __fadd_rn(y[i], rr[i]);
      bad = !(fabs((double)v - (double)xv) <= e) || tier_rank(iso, v) != tier_rank(iso, xv);
      y[i] = bad ? xv : v;
    }
    const unsigned long long m = __ballot(bad);
    if (lane_id() == 0) {
      const uint64_t w = i / 64;
      mask[w] = m;
      cnt[w] = (uint64_t)__popcll(m);
    }
  }
}

// The current tier's place in the container (one thread): offsets, the
// record, the cursor, the status, and the zero padding of its parts.
__global__ void k_tier_place(TierState *S, int t, double e, const chr_result *res, const int32_t *dstatus,
                             const uint64_t *pre, uint64_t nw, uint8_t *out, uint64_t cap) {
  if (threadIdx.x != 0) return;
  const uint64_t sb = res->stream_bytes;
  if (S->status == 0 && res->status != 0) S->status = res->status;
  if (S->status == 0 && *dstatus != 0) S->status = CHR_E_CORRUPT;
  const uint64_t nc = t == 0 ? 0 : pre[nw];
  const uint64_t so = S->cursor, io = tpad8(so + sb), vo = tpad8(io + 8 * nc), nx = tpad8(vo + 4 * nc);
  S->so = so; S->sb = sb; S->nc = nc; S->io = io; S->vo = vo;
  uint64_t *rc = S->rec[t];
  double ev = e;
  uint64_t eb;
  __builtin_memcpy(&eb, &ev, 8);
  rc[0] = eb; rc[1] = so; rc[2] = sb; rc[3] = nc; rc[4] = io; rc[5] = vo; rc[6] = 0; rc[7] = 0;
  S->cursor = nx;
  if (S->status == 0 && nx > cap) S->status = CHR_E_CAPACITY;
  if (S->status == 0) {
    for (uint64_t b = so + sb; b < io; b++) out[b] = 0;
    for (uint64_t b = vo + 4 * nc; b < nx; b++) out[b] = 0;
  }
}

// The tier's stream into the container (8 bytes per thread; a CHR stream is
// a multiple of 8 bytes long, the tail is handled anyway).
__global__ __launch_bounds__(kBS) void k_tier_copy(const TierState *S, const uint8_t *__restrict__ B,
                                                    uint8_t *__restrict__ out) {
  if (S->status != 0) return;
  const uint64_t so = S->so, sb = S->sb;
  const uint64_t n8 = sb / 8;
  const uint64_t *src = reinterpret_cast<const uint64_t *>(B);
  uint64_t *dst = reinterpret_cast<uint64_t *>(out + so);
  for (uint64_t i = (uint64_t)blockIdx.x * kBS + threadIdx.x; i < n8; i += (uint64_t)gridDim.x * kBS) dst[i] = src[i];
  if (blockIdx.x == 0)
    for (uint64_t b = 8 * n8 + threadIdx.x; b < sb; b += kBS) out[so + b] = B[b];
}

// The tier's corrections in index order (one thread per 64-point word; the
// words without a correction, nearly all of them, cost one load).
__global__ __launch_bounds__(kBS) void k_tier_corr(const TierState *S, const unsigned long long *__restrict__ mask,
                                                    const uint64_t *__restrict__ pre, const float *__restrict__ x,
                                                    uint64_t nw, uint8_t *__restrict__ out) {
  if (S->status != 0) return;
  uint64_t *idx = reinterpret_cast<uint64_t *>(out + S->io);
  float *val = reinterpret_cast<float *>(out + S->vo);
  for (uint64_t w = (uint64_t)blockIdx.x * kBS + threadIdx.x; w < nw; w += (uint64_t)gridDim.x * kBS) {
    unsigned long long m = mask[w];
    uint64_t pos = m ? pre[w] : 0;
    while (m) {
      const uint64_t i = 64 * w + (uint64_t)(__ffsll((long long)m) - 1);
      idx[pos] = i;
      val[pos] = x[i];
      pos++;
      m &= m - 1;
    }
  }
}

// Header and tier records; the result.
__global__ void k_tier_finish(const TierState *S, TierHead h, uint8_t *out, uint64_t *result) {
  const uint64_t total = S->cursor;
  const int64_t st = S->status;
  if (threadIdx.x == 0) {
    result[0] = total;
    result[1] = (uint64_t)st;
  }
  if (st != 0) return;
  uint32_t *o32 = reinterpret_cast<uint32_t *>(out);
  uint64_t *o64 = reinterpret_cast<uint64_t *>(out);
  for (uint32_t i = threadIdx.x; i < kTHead / 4; i += blockDim.x) {
    uint32_t v = 0;
    if (i == 0) v = kTMagic;
    if (i == 1) v = 1u;
    if (i == 2) v = (uint32_t)h.T;
    if (i == 3) v = (uint32_t)h.K;
    if (i >= 4 && i < 10) v = (uint32_t)((uint64_t)h.dims[(i - 4) / 2] >> (32 * ((i - 4) & 1)));
    if (i == 10) v = (uint32_t)h.levels;
    if (i == 11) v = (uint32_t)h.block;
    if (i == 12) v = (uint32_t)h.qmax;
    if (i >= 14 && i < 30) v = __float_as_uint(h.iso[i - 14]);
    if (i == 30) v = (uint32_t)total;
    if (i == 31) v = (uint32_t)(total >> 32);
    o32[i] = v;
  }
  for (uint32_t i = threadIdx.x; i < CHR_MAX_TIERS * 8; i += blockDim.x) {
    const uint32_t t = i / 8;
    o64[kTHead / 8 + i] = (int)t < h.T ? S->rec[t][i % 8] : 0ull;
  }
}

__global__ __launch_bounds__(kBS) void k_tier_add(float *__restrict__ out, const float *__restrict__ r, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * kBS + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kBS)
    out[i] = __fadd_rn(out[i], r[i]);
}

__global__ __launch_bounds__(kBS) void k_tier_apply(const uint8_t *__restrict__ in, uint64_t io, uint64_t vo,
                                                     uint64_t nc, float *__restrict__ out, uint64_t n,
                                                     int32_t *status) {
  for (uint64_t j = (uint64_t)blockIdx.x * kBS + threadIdx.x; j < nc; j += (uint64_t)gridDim.x * kBS) {
    const uint64_t i = reinterpret_cast<const uint64_t *>(in + io)[j];
    if (i >= n) {
      *status = CHR_E_CORRUPT;
      continue;
    }
    out[i] = reinterpret_cast<const float *>(in + vo)[j];
  }
}

unsigned grid_for(uint64_t n, uint64_t per_block) {
  const uint64_t g = (n + per_block - 1) / per_block;
  return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(g, 1u << 20));
}

struct TierLayout {
  size_t y, r, B, cws, dws, res, st, mask, cnt, pre, tmp, state, total;
  size_t Bbytes, cwsbytes, dwsbytes;
};

bool tier_layout(const int64_t dims[3], const chr_params *p, TierLayout &Lo, std::string &why) {
  chr_params q = *p;
  q.error_bound_far = 0.0;
  const size_t sb = chr_compress_bound(dims, &q);
  const size_t cw = enc_workspace_bytes(dims, &q);
  if (sb == 0 || cw == 0) { why = "bad parameters for these dims"; return false; }
  Geo g;
  uint64_t poff = 0;
  if (enc_geometry(dims, 0.0, nullptr, 0, &q, g, poff)) { why = "bad parameters for these dims"; return false; }
  const uint64_t N = (uint64_t)dims[0] * dims[1] * dims[2], nw = (N + 63) / 64;
  auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
  size_t o = 0;
  Lo.y = o; o = al(o + 4 * N);
  Lo.r = o; o = al(o + 4 * N);
  Lo.B = o; Lo.Bbytes = sb; o = al(o + sb);
  Lo.cws = o; Lo.cwsbytes = cw; o = al(o + cw);
  Lo.dwsbytes = dec_workspace_bytes(g, 0);
  Lo.dws = o; o = al(o + std::max<size_t>(Lo.dwsbytes, 256));
  Lo.res = o; o = al(o + sizeof(chr_result));
  Lo.st = o; o = al(o + 4);
  Lo.mask = o; o = al(o + 8 * nw);
  Lo.cnt = o; o = al(o + 8 * nw);
  Lo.pre = o; o = al(o + 8 * (nw + 1));
  Lo.tmp = o; o = al(o + 8 * (size_t)scan_tmp_elems((int64_t)nw));
  Lo.state = o; o = al(o + sizeof(TierState));
  Lo.total = o;
  return true;
}

bool bounds_ok(const double *b, int T) {
  if (T < 1 || T > CHR_MAX_TIERS || !b) return false;
  for (int t = 0; t < T; t++) {
    if (!(b[t] >= 0) || !std::isfinite(b[t])) return false;
    if (t > 0 && !(b[t] < b[t - 1])) return false;
  }
  return true;
}

}  // namespace
}  // namespace chr

using namespace chr;

extern "C" {

size_t chr_tiers_bound(const int64_t dims[3], int n_tiers, const chr_params *p) {
  if (!dims || !p || n_tiers < 1 || n_tiers > CHR_MAX_TIERS) { api_fail(CHR_E_INVAL, "bad argument"); return 0; }
  chr_params q = *p;
  q.error_bound_far = 0.0;
  const size_t sb = chr_compress_bound(dims, &q);
  if (sb == 0) return 0;
  const uint64_t N = (uint64_t)dims[0] * dims[1] * dims[2];
  return (size_t)(kTData + (uint64_t)n_tiers * (tpad8(sb) + 8 * N + tpad8(4 * N)));
}

size_t chr_tiers_workspace(const int64_t dims[3], const chr_params *p) {
  if (!dims || !p) { api_fail(CHR_E_INVAL, "NULL argument"); return 0; }
  TierLayout Lo;
  std::string why;
  if (!tier_layout(dims, p, Lo, why)) { api_fail(CHR_E_INVAL, why); return 0; }
  return Lo.total;
}

int chr_tiers_compress(const float *d_field, const int64_t dims[3], const double *h_bounds, int n_tiers,
                       const float *h_isovalues, int n_iso, const chr_params *p, void *d_out, size_t capacity,
                       uint64_t *d_result, void *d_ws, size_t ws_bytes, void *stream) {
  if (!d_field || !dims || !p || !d_out || !d_result || !d_ws) return api_fail(CHR_E_INVAL, "NULL argument");
  if (!bounds_ok(h_bounds, n_tiers))
    return api_fail(CHR_E_INVAL, "tier bounds: 1..8 finite values >= 0, strictly decreasing");
  if (p->error_bound_far != 0) return api_fail(CHR_E_INVAL, "tiers take one bound per tier (error_bound_far = 0)");
  if ((reinterpret_cast<uintptr_t>(d_out) & 7) || (reinterpret_cast<uintptr_t>(d_result) & 7))
    return api_fail(CHR_E_INVAL, "container and result must be 8-byte aligned");
  TierLayout Lo;
  std::string why;
  if (!tier_layout(dims, p, Lo, why)) return api_fail(CHR_E_INVAL, why);
  if (ws_bytes < Lo.total) return api_fail(CHR_E_NOMEM, "workspace too small: need " + std::to_string(Lo.total));
  if (capacity < (size_t)kTData) return api_fail(CHR_E_CAPACITY, "capacity below the container header");
  hipStream_t s = static_cast<hipStream_t>(stream);
  uint8_t *ws = static_cast<uint8_t *>(d_ws);
  float *y = reinterpret_cast<float *>(ws + Lo.y), *r = reinterpret_cast<float *>(ws + Lo.r);
  uint8_t *B = ws + Lo.B;
  chr_result *res = reinterpret_cast<chr_result *>(ws + Lo.res);
  int32_t *dst = reinterpret_cast<int32_t *>(ws + Lo.st);
  unsigned long long *mask = reinterpret_cast<unsigned long long *>(ws + Lo.mask);
  uint64_t *cnt = reinterpret_cast<uint64_t *>(ws + Lo.cnt), *pre = reinterpret_cast<uint64_t *>(ws + Lo.pre);
  uint64_t *tmp = reinterpret_cast<uint64_t *>(ws + Lo.tmp);
  TierState *S = reinterpret_cast<TierState *>(ws + Lo.state);
  uint8_t *out = static_cast<uint8_t *>(d_out);
  const uint64_t N = (uint64_t)dims[0] * dims[1] * dims[2], nw = (N + 63) / 64;
  chr_params q = *p;
  int ecpw, dcpw;
  current_tiles(ecpw, dcpw);
  TierHead h{};
  k_tier_init<<<1, kBS, 0, s>>>(S);
  for (int t = 0; t < n_tiers; t++) {
    if (t > 0) k_tier_residual<<<grid_for(N, kBS), kBS, 0, s>>>(d_field, y, r, N);
    EncJob J;
    int rc = enc_prepare(t == 0 ? d_field : r, dims, h_bounds[t], t == 0 ? h_isovalues : nullptr, t == 0 ? n_iso : 0,
                         &q, B, Lo.Bbytes, res, nullptr, nullptr, ws + Lo.cws, Lo.cwsbytes, ecpw, J);
    if (rc) return rc;
    if (t == 0) {
      h.T = n_tiers;
      h.K = J.P.g.K;
      h.levels = p->levels;
      h.block = p->block;
      h.qmax = p->qmax;
      for (int a = 0; a < 3; a++) h.dims[a] = dims[a];
      for (int j = 0; j < 16; j++) h.iso[j] = J.P.g.iso[j];
    }
    launch_encode(J.P, 0, J.scan, J.scan64, s);
    DecJob D;
    rc = dec_prepare(J.P.g, J.P.payload_off, 0, B, Lo.Bbytes, t == 0 ? y : r, dst, ws + Lo.dws, Lo.dwsbytes, dcpw, D);
    if (rc) return rc;
    launch_status_reset(dst, s);
    launch_decode(D.D, s);
    if (t > 0) {
      TierIso iso{};
      iso.K = h.K;
      for (int j = 0; j < 16; j++) iso.v[j] = h.iso[j];
      k_tier_combine<<<grid_for(nw * 64, kBS), kBS, 0, s>>>(d_field, y, r, N, h_bounds[t], iso, mask, cnt);
      scan_u64(cnt, pre, (int64_t)nw, tmp, s);
    }
    k_tier_place<<<1, 64, 0, s>>>(S, t, h_bounds[t], res, dst, pre, nw, out, capacity);
    // grid-stride copy over the stream's actual size (read on the device)
    k_tier_copy<<<std::min<unsigned>(grid_for(Lo.Bbytes / 8, kBS), 4096u), kBS, 0, s>>>(S, B, out);
    if (t > 0) k_tier_corr<<<grid_for(nw, kBS), kBS, 0, s>>>(S, mask, pre, d_field, nw, out);
  }
  k_tier_finish<<<1, kBS, 0, s>>>(S, h, out, d_result);
  return api_check_launch("chr_tiers_compress");
}

int chr_tiers_header(const void *h_head, size_t head_bytes, chr_tier_header *o) {
  if (!h_head || !o) return api_fail(CHR_E_INVAL, "NULL argument");
  const uint8_t *c = static_cast<const uint8_t *>(h_head);
  auto g32 = [&](size_t off) { uint32_t v; std::memcpy(&v, c + off, 4); return v; };
  auto g64 = [&](size_t off) { uint64_t v; std::memcpy(&v, c + off, 8); return v; };
  if (head_bytes < (size_t)kTData || g32(0) != kTMagic || g32(4) != 1u)
    return api_fail(CHR_E_CORRUPT, "not a tier container (magic/version)");
  std::memset(o, 0, sizeof(*o));
  o->n_tiers = (int)g32(8);
  o->n_iso = (int)g32(12);
  for (int a = 0; a < 3; a++) o->dims[a] = (int64_t)g64(16 + 8 * a);
  o->levels = (int)g32(40);
  o->block = (int)g32(44);
  o->qmax = (int)g32(48);
  for (int j = 0; j < 16; j++) std::memcpy(&o->isovalues[j], c + 56 + 4 * j, 4);
  o->total_bytes = g64(120);
  if (o->n_tiers < 1 || o->n_tiers > CHR_MAX_TIERS || o->n_iso < 0 || o->n_iso > 16)
    return api_fail(CHR_E_CORRUPT, "tier container: bad tier or isovalue count");
  for (int t = 0; t < o->n_tiers; t++) {
    const size_t r = kTHead + kTRec * (size_t)t;
    std::memcpy(&o->bound[t], c + r, 8);
    o->stream_offset[t] = g64(r + 8);
    o->stream_bytes[t] = g64(r + 16);
    o->n_corrections[t] = g64(r + 24);
    o->index_offset[t] = g64(r + 32);
    o->value_offset[t] = g64(r + 40);
    if ((o->stream_offset[t] | o->index_offset[t] | o->value_offset[t]) & 7 ||
        o->stream_offset[t] + o->stream_bytes[t] > o->total_bytes ||
        o->index_offset[t] + 8 * o->n_corrections[t] > o->total_bytes ||
        o->value_offset[t] + 4 * o->n_corrections[t] > o->total_bytes)
      return api_fail(CHR_E_CORRUPT, "tier container: record out of range");
  }
  if (!bounds_ok(o->bound, o->n_tiers)) return api_fail(CHR_E_CORRUPT, "tier container: bad bounds");
  chr_params p{o->levels, o->block, o->qmax, 0.0};
  if (chr_compress_bound(o->dims, &p) == 0) return api_fail(CHR_E_CORRUPT, "tier container: bad parameters");
  return CHR_OK;
}

size_t chr_tiers_reconstruct_workspace(const chr_tier_header *h) {
  if (!h) { api_fail(CHR_E_INVAL, "NULL argument"); return 0; }
  chr_params p{h->levels, h->block, h->qmax, 0.0};
  Geo g;
  uint64_t poff;
  if (enc_geometry(h->dims, 0.0, nullptr, 0, &p, g, poff)) return 0;
  const uint64_t N = (uint64_t)h->dims[0] * h->dims[1] * h->dims[2];
  return ((4 * N + 255) & ~(uint64_t)255) + std::max<size_t>(dec_workspace_bytes(g, 0), 256);
}

int chr_tiers_reconstruct(const chr_tier_header *h, const void *d_container, size_t bytes, double error_bound,
                          float *d_out, int32_t *d_status, void *d_ws, size_t ws_bytes, int *tier_used, void *stream) {
  if (!h || !d_container || !d_out || !d_status || !d_ws) return api_fail(CHR_E_INVAL, "NULL argument");
  if (reinterpret_cast<uintptr_t>(d_container) & 7) return api_fail(CHR_E_INVAL, "container must be 8-byte aligned");
  if (!bounds_ok(h->bound, h->n_tiers)) return api_fail(CHR_E_INVAL, "bad tier header");
  if (bytes < h->total_bytes) return api_fail(CHR_E_CORRUPT, "container shorter than its header states");
  int use = -1;
  for (int t = 0; t < h->n_tiers; t++)
    if (h->bound[t] <= error_bound) { use = t; break; }
  if (use < 0) return api_fail(CHR_E_ACCURACY, "no tier meets the requested error bound");
  const size_t need = chr_tiers_reconstruct_workspace(h);
  if (need == 0) return api_fail(CHR_E_INVAL, "bad tier header parameters");
  if (ws_bytes < need) return api_fail(CHR_E_NOMEM, "workspace too small: need " + std::to_string(need));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const uint64_t N = (uint64_t)h->dims[0] * h->dims[1] * h->dims[2];
  uint8_t *ws = static_cast<uint8_t *>(d_ws);
  float *r = reinterpret_cast<float *>(ws);
  uint8_t *dws = ws + ((4 * N + 255) & ~(uint64_t)255);
  const uint8_t *c = static_cast<const uint8_t *>(d_container);
  chr_params p{h->levels, h->block, h->qmax, 0.0};
  int ecpw, dcpw;
  current_tiles(ecpw, dcpw);
  launch_status_reset(d_status, s);
  for (int t = 0; t <= use; t++) {
    Geo g;
    uint64_t poff;
    int rc = enc_geometry(h->dims, h->bound[t], t == 0 ? h->isovalues : nullptr, t == 0 ? h->n_iso : 0, &p, g, poff);
    if (rc) return rc;
    DecJob D;
    rc = dec_prepare(g, poff, 0, c + h->stream_offset[t], h->stream_bytes[t], t == 0 ? d_out : r, d_status, dws,
                     ws_bytes - (size_t)(dws - ws), dcpw, D);
    if (rc) return rc;
    launch_decode(D.D, s);
    if (t > 0) {
      k_tier_add<<<grid_for(N, kBS), kBS, 0, s>>>(d_out, r, N);
      if (h->n_corrections[t])
        k_tier_apply<<<grid_for(h->n_corrections[t], kBS), kBS, 0, s>>>(c, h->index_offset[t], h->value_offset[t],
                                                                         h->n_corrections[t], d_out, N, d_status);
    }
  }
  if (tier_used) *tier_used = use;
  return api_check_launch("chr_tiers_reconstruct");
}

}  // extern "C"
