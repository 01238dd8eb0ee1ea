// capi.hip -- the C ABI (include/chr.h): argument checks, plans, workspace
// layouts and host-side stream parsing.  All compute runs in the kernels of
// encode.hip, decode.hip, mc.hip and scan.hip.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "capi_internal.h"

using namespace chr;

namespace {

thread_local std::string g_err;

// Tile shapes of the level-0 kernels (work distribution only; results do not
// depend on them).  Set by chr_set_tiles, or per batch by its autotuner.
struct Tune {
  int enc_cpw0 = 8;
  int dec_cpw0 = 16;
  int tile0 = 1;   // level 0 of 64-cell blocks by plane pairs
} g_tune;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

bool dims_ok(const int64_t d[3]) {
  if (!d) return false;
  for (int a = 0; a < 3; a++)
    if (d[a] < 1 || d[a] > ((int64_t)1 << 30)) return false;
  return true;
}

size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

// Per-axis block extents: (cells of the block, how many blocks have it).
struct AxisClass {
  int64_t ext[2];
  int64_t count[2];
  int n;
};

AxisClass axis_classes(int64_t n, int64_t B) {
  AxisClass c{};
  int64_t cells = n - 1;
  int64_t nb = blocks_along(n, B);
  if (cells <= 0) {
    c.ext[0] = 0; c.count[0] = 1; c.n = 1;
    return c;
  }
  int64_t last = cells - (nb - 1) * B;
  if (last == B) { c.ext[0] = B; c.count[0] = nb; c.n = 1; }
  else {
    c.n = 0;
    if (nb > 1) { c.ext[c.n] = B; c.count[c.n] = nb - 1; c.n++; }
    c.ext[c.n] = last; c.count[c.n] = 1; c.n++;
  }
  return c;
}

bool params_ok(const int64_t dims[3], const chr_params *p, std::string &why) {
  if (!dims_ok(dims)) { why = "dims must be in [1, 2^30]"; return false; }
  if (!p) { why = "params is NULL"; return false; }
  if (p->levels < 1 || p->levels > kMaxLevels) { why = "levels must be in [1, 16]"; return false; }
  int64_t S = (int64_t)1 << (p->levels - 1);
  if (p->block < 1 || p->block % S) { why = "block must be a positive multiple of 2^(levels-1)"; return false; }
  if (p->qmax < 1 || p->qmax > 32767) { why = "qmax must be in [1, 32767]"; return false; }
  // every section's point count must fit 31 bits
  int64_t e[3];
  for (int a = 0; a < 3; a++) e[a] = std::min<int64_t>(p->block, dims[a] - 1) + 1;
  if ((double)e[0] * (double)e[1] * (double)e[2] >= 2147483647.0) { why = "block too large for this field"; return false; }
  if (p->merge < 0 || p->merge > 16) { why = "merge must be in [0, 16]"; return false; }
  if (p->merge > 1) {
    for (int a = 0; a < 3; a++) e[a] = std::min<int64_t>((int64_t)p->merge * p->block, dims[a] - 1) + 1;
    if ((double)e[0] * (double)e[1] * (double)e[2] >= 2147483647.0) {
      why = "merged units too large for this field";
      return false;
    }
    if (p->error_bound_far != 0) { why = "merging is not combined with differentiated error control"; return false; }
  }
  return true;
}

void fill_geo(Geo &g, const int64_t dims[3], int nL, int B, int qmax) {
  std::memset(&g, 0, sizeof(g));
  for (int a = 0; a < 3; a++) {
    g.n[a] = dims[a];
    g.nb[a] = blocks_along(dims[a], B);
  }
  g.nblocks = g.nb[0] * g.nb[1] * g.nb[2];
  g.nL = nL;
  g.B = B;
  g.qmax = qmax;
}

void set_quant(Geo &g, double e) {
  g.e = e;
  g.inv = 0.f;
  g.step = 0.f;
  if (e > 0) {
    g.inv = (float)(1.0 / (2.0 * e));
    g.step = (float)(2.0 * e);
  }
  g.lossless = (!(e > 0) || g.step == 0.0f || !std::isfinite(g.step)) ? 1 : 0;
  // fl(d) = d (1 + r) with |r| <= 2^-24, so |fl(d)| <= e (1 - 2^-23) gives
  // |d| <= e (1 - 2^-23) / (1 - 2^-24) < e; rounded down to binary32
  g.ein = 0.f;
  if (e > 0) {
    const double t = e * (1.0 - 0x1p-23);
    float f = (float)t;
    if ((double)f > t) f = std::nextafter(f, 0.0f);
    g.ein = f;
  }
}

// The far quantizer of differentiated error control (same rule as set_quant).
void set_quant_far(Geo &g, double e2) {
  Geo t = g;
  set_quant(t, e2);
  g.diff = 1;
  g.e2 = t.e;
  g.inv2 = t.inv;
  g.step2 = t.step;
  g.lossless2 = t.lossless;
}

// Merging parameter of a geometry (0 and 1: none).
void set_merge(Geo &g, int merge) {
  g.merge = merge > 1 ? merge : 1;
  for (int a = 0; a < 3; a++) g.mb[a] = g.merge;
}

// max chunks of a level-l section (the first block is the largest)
uint32_t max_chunks(const Geo &g, int l) {
  int64_t o[3], hi[3];
  block_ext(g, 0, o, hi);
  Sec s = sec_geom(o, hi, l, g.nL - 1);
  return (s.npts + 63) / 64;
}

struct EncLayout {
  size_t off_G, off_cnt, off_P, off_scan, off_pay, off_emask, off_exv, off_part, off_bst, off_csum, off_secsz, off_secoff,
      off_scan64, off_act, off_units, off_ubase, total, part_records;
};

EncLayout enc_layout(EncPlan &P) {
  const Geo &g = P.g;
  const int L = g.nL - 1;
  int64_t base = 0;
  for (int l = L; l >= 0; l--) {
    P.maxch[l] = max_chunks(g, l);
    P.slot_base[l] = base;
    base += g.nblocks * (int64_t)P.maxch[l];
  }
  P.nslots = base;
  if (g.merge > 1) {
    // merged units: no more points than their blocks, at most one partial
    // chunk per unit and level beyond them; workgroups per unit sized for
    // the largest possible unit (merge blocks per axis)
    P.nslots += g.nblocks * g.nL;
    int64_t o[3], hi[3];
    largest_ext(g, o, hi);
    for (int l = L; l >= 0; l--) P.maxch[l] = (uint32_t)((sec_geom(o, hi, l, L).npts + 63) / 64);
  }
  int64_t goff = 0;
  for (int l = 0; l < kMaxLevels; l++) {
    for (int a = 0; a < 3; a++) P.gd[l][a] = (l <= L) ? lvl_dim(g.n[a], l) : 0;
    P.g_off[l] = 0;
    if (l >= 1 && l <= L) {
      P.g_off[l] = goff;
      goff += P.gd[l][0] * P.gd[l][1] * P.gd[l][2];
    }
  }
  const int64_t nsec = g.nblocks * g.nL;
  P.payload_off = kHeaderBytes + 16 * (uint64_t)nsec + 16 * (uint64_t)g.nblocks;
  EncLayout Lo{};
  size_t o = 0;
  Lo.off_G = o; o = align256(o + sizeof(float) * (size_t)std::max<int64_t>(goff, 1));
  Lo.off_cnt = o; o = align256(o + sizeof(U4) * (size_t)P.nslots);
  Lo.off_P = o; o = align256(o + sizeof(U4) * (size_t)(P.nslots + 1));
  Lo.off_scan = o; o = align256(o + sizeof(U4) * (size_t)scan_tmp_elems(P.nslots));
  Lo.off_pay = o; o = align256(o + sizeof(uint32_t) * 32 * (size_t)P.nslots);
  Lo.off_emask = o; o = align256(o + sizeof(uint64_t) * (size_t)P.nslots);
  Lo.off_exv = o; o = align256(o + sizeof(float) * 64 * (size_t)P.nslots);
  P.part_l1 = encode_fine_groups(P);
  P.part_l2 = P.part_l1 + encode_l1_groups(P);
  P.part_per_block = P.part_l2 + encode_l2_groups(P) + 1;
  P.l2fast = encode_l2_fast(P) ? 1 : 0;
  {
    // workspace sized for the finest level-0 tiling of either level-0 path
    EncPlan q = P;
    q.cpw0 = 1;
    q.tile0 = 0;
    const int64_t ppb_chunks = encode_fine_groups(q);
    q.tile0 = 1;
    const int64_t ppb0 = std::max<int64_t>(ppb_chunks, encode_fine_groups(q));
    q.tile1 = 0;
    const int64_t ppb1_chunks = encode_l1_groups(q);
    q.tile1 = 1;
    const int64_t ppb1 = std::max<int64_t>(ppb1_chunks, encode_l1_groups(q));
    q.top = 0;
    const int64_t ppb_max = ppb0 + ppb1 + encode_l2_groups(q) + 1;
    Lo.part_records = (size_t)(g.nblocks * ppb_max);
  }
  encode_pack_layout(P);
  Lo.off_part = o; o = align256(o + sizeof(Part) * Lo.part_records);
  Lo.off_bst = o; o = align256(o + sizeof(Part) * (size_t)g.nblocks);
  Lo.off_csum = o; o = align256(o + sizeof(uint32_t) * kSumSegs * (size_t)(g.nblocks + 1));
  Lo.off_secsz = o; o = align256(o + sizeof(uint64_t) * (size_t)nsec);
  Lo.off_secoff = o; o = align256(o + sizeof(uint64_t) * (size_t)(nsec + 1));
  Lo.off_scan64 = o; o = align256(o + sizeof(uint64_t) * (size_t)scan_tmp_elems(nsec));
  // activity flags (or index signatures), then 16 partial (min, max) key
  // pairs per block
  Lo.off_act = o; o = align256(o + sizeof(uint32_t) * (size_t)g.nblocks * (1 + 2 * kActSplit));
  if (g.merge > 1) {
    // merged units: their boxes and first slots
    Lo.off_units = o; o = align256(o + sizeof(uint32_t) * 8 * (size_t)g.nblocks);
    Lo.off_ubase = o; o = align256(o + sizeof(int64_t) * (size_t)nsec);
  }
  Lo.total = o;
  return Lo;
}

int prepare_iso(const float *h_iso, int n_iso, Geo &g, std::string &why) {
  if (n_iso < 0 || n_iso > kMaxIso) { why = "n_iso must be in [0, 16]"; return -1; }
  if (n_iso > 0 && !h_iso) { why = "isovalues is NULL"; return -1; }
  float t[kMaxIso];
  for (int j = 0; j < n_iso; j++) {
    if (!std::isfinite(h_iso[j])) { why = "isovalues must be finite"; return -1; }
    t[j] = h_iso[j];
  }
  std::sort(t, t + n_iso);
  int k = 0;
  for (int j = 0; j < n_iso; j++)
    if (k == 0 || t[j] != g.iso[k - 1]) g.iso[k++] = t[j];
  for (int j = k; j < kMaxIso; j++) g.iso[j] = 0.f;
  g.K = k;
  return 0;
}

uint32_t host_checksum(const uint8_t *p, size_t nbytes) {
  uint32_t s = 0;
  for (size_t j = 0; j < nbytes / 4; j++) {
    uint32_t w;
    std::memcpy(&w, p + 4 * j, 4);
    s += fmix32(w ^ (uint32_t)((uint32_t)j * 0x9E3779B9u));
  }
  return s;
}

template <class T>
T rd(const uint8_t *p) {
  T v;
  std::memcpy(&v, p, sizeof(T));
  return v;
}

int check_hip(const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(CHR_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return CHR_OK;
}

struct Prof {
  std::string name;
  std::vector<hipEvent_t> ev;  // begin/end pairs
  int used = 0;                // events recorded
  bool on = false;
} g_prof;

}  // namespace

namespace chr {
int api_fail(int code, const std::string &msg) { return fail(code, msg); }
int api_check_launch(const char *what) { return check_hip(what); }
void current_tiles(int &enc_cpw, int &dec_cpw) {
  enc_cpw = g_tune.enc_cpw0;
  dec_cpw = g_tune.dec_cpw0;
}

bool tiles_ok(int enc_cpw, int dec_cpw) {
  const bool e = enc_cpw == 1 || enc_cpw == 2 || enc_cpw == 4 || enc_cpw == 8 || enc_cpw == 16;
  const bool d = dec_cpw == 8 || dec_cpw == 16 || dec_cpw == 32 || dec_cpw == 64;
  return e && d;
}

size_t enc_workspace_bytes(const int64_t dims[3], const chr_params *p) {
  std::string why;
  if (!params_ok(dims, p, why)) { g_err = why; return 0; }
  EncPlan P;
  std::memset(&P, 0, sizeof(P));
  P.cpw0 = 4;
  fill_geo(P.g, dims, p->levels, p->block, p->qmax);
  set_merge(P.g, p->merge);
  return enc_layout(P).total;
}

int enc_geometry(const int64_t dims[3], double error_bound, const float *h_iso, int n_iso, const chr_params *p,
                 Geo &g, uint64_t &payload_off) {
  std::string why;
  if (!params_ok(dims, p, why)) return fail(CHR_E_INVAL, why);
  if (!(error_bound >= 0) || !std::isfinite(error_bound)) return fail(CHR_E_INVAL, "error_bound must be finite and >= 0");
  const double far = p->error_bound_far;
  if (far != 0 && !(far >= error_bound && std::isfinite(far)))
    return fail(CHR_E_INVAL, "error_bound_far must be 0 or finite and >= error_bound");
  fill_geo(g, dims, p->levels, p->block, p->qmax);
  if (prepare_iso(h_iso, n_iso, g, why)) return fail(CHR_E_INVAL, why);
  set_quant(g, error_bound);
  if (far != 0) set_quant_far(g, far);
  if (g.nblocks > 65535) return fail(CHR_E_INVAL, "more than 65535 blocks: use a larger block");
  payload_off = kHeaderBytes + 16 * (uint64_t)g.nblocks * g.nL + 16 * (uint64_t)g.nblocks;
  return CHR_OK;
}

int enc_prepare(const float *d_field, const int64_t dims[3], double error_bound, const float *h_iso, int n_iso,
                const chr_params *p, void *d_stream, size_t capacity, chr_result *d_result, int32_t *d_codes,
                uint8_t *d_flags, void *d_ws, size_t ws_bytes, int cpw0, EncJob &J, bool merging) {
  if (!d_field || !d_stream || !d_result || !d_ws) return fail(CHR_E_INVAL, "NULL device pointer");
  if (p && p->merge > 1 && !merging) return fail(CHR_E_INVAL, "block merging is available through chr_compress only");
  if (reinterpret_cast<uintptr_t>(d_stream) & 7) return fail(CHR_E_INVAL, "stream buffer must be 8-byte aligned");
  EncPlan &P = J.P;
  std::memset(&P, 0, sizeof(P));
  uint64_t poff = 0;
  int rc = enc_geometry(dims, error_bound, h_iso, n_iso, p, P.g, poff);
  if (rc) return rc;
  P.cpw0 = cpw0;
  make_l0geo(P.g, P.l0);
  set_merge(P.g, p->merge);
  if (P.g.merge > 1) P.l0.small = 0;   // units of varying shapes: the general kernels
  P.codes = d_codes;
  P.flags = d_flags;
  P.tile0 = (g_tune.tile0 && encode_tile0_ok(P)) ? 1 : 0;
  P.tile1 = (g_tune.tile0 && encode_tile1_ok(P)) ? 1 : 0;
  P.top = (g_tune.tile0 && encode_top_ok(P)) ? 1 : 0;
  EncLayout Lo = enc_layout(P);
  if (ws_bytes < Lo.total) return fail(CHR_E_NOMEM, "workspace too small: need " + std::to_string(Lo.total));
  if (capacity < P.payload_off) return fail(CHR_E_CAPACITY, "capacity below the header and tables");
  uint8_t *ws = static_cast<uint8_t *>(d_ws);
  P.x = d_field;
  P.G = reinterpret_cast<float *>(ws + Lo.off_G);
  P.cnt = reinterpret_cast<U4 *>(ws + Lo.off_cnt);
  P.P = reinterpret_cast<U4 *>(ws + Lo.off_P);
  P.pay = reinterpret_cast<uint32_t *>(ws + Lo.off_pay);
  P.emask = reinterpret_cast<unsigned long long *>(ws + Lo.off_emask);
  P.exv = reinterpret_cast<float *>(ws + Lo.off_exv);
  P.part = reinterpret_cast<Part *>(ws + Lo.off_part);
  P.bst = reinterpret_cast<Part *>(ws + Lo.off_bst);
  P.csum = reinterpret_cast<uint32_t *>(ws + Lo.off_csum);
  P.secsz = reinterpret_cast<uint64_t *>(ws + Lo.off_secsz);
  P.secoff = reinterpret_cast<uint64_t *>(ws + Lo.off_secoff);
  P.out = static_cast<uint8_t *>(d_stream);
  P.cap = capacity;
  P.result = d_result;
  P.codes = d_codes;
  P.flags = d_flags;
  P.act = reinterpret_cast<uint32_t *>(ws + Lo.off_act);
  J.scan = reinterpret_cast<U4 *>(ws + Lo.off_scan);
  J.scan64 = reinterpret_cast<uint64_t *>(ws + Lo.off_scan64);
  if (P.g.merge > 1) {
    J.units = reinterpret_cast<uint32_t *>(ws + Lo.off_units);
    J.ubase = reinterpret_cast<int64_t *>(ws + Lo.off_ubase);
  }
  return CHR_OK;
}

// Block merging before compression: the blocks' index signatures computed
// on the device, the units laid out here (greedy, lexicographic block order:
// a unit grows along x while the next block is free and has its signature,
// then along y by whole rows, then along z by whole planes, up to `merge`
// blocks per axis), and the plan switched from blocks to units.  Waits for
// the stream once.
int enc_merge_units(EncJob &J, hipStream_t s) {
  EncPlan &P = J.P;
  const Geo gb = P.g;
  const int64_t nb0 = gb.nb[0], nb1 = gb.nb[1], nb2 = gb.nb[2], nblk = gb.nblocks;
  const int M = gb.merge, L = gb.nL - 1;
  launch_block_signatures(P, s);
  std::vector<uint32_t> sig((size_t)nblk);
  if (hipMemcpyAsync(sig.data(), P.act, sizeof(uint32_t) * (size_t)nblk, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(CHR_E_HIP, "block signatures: copy to the host failed");
  std::vector<int32_t> unit((size_t)nblk, -1);
  std::vector<uint32_t> box;
  auto at = [&](int64_t z, int64_t y, int64_t x) { return (size_t)((z * nb1 + y) * nb2 + x); };
  auto free_same = [&](int64_t z, int64_t y, int64_t x, uint32_t g) { return unit[at(z, y, x)] < 0 && sig[at(z, y, x)] == g; };
  for (int64_t z = 0; z < nb0; z++)
    for (int64_t y = 0; y < nb1; y++)
      for (int64_t x = 0; x < nb2; x++) {
        if (unit[at(z, y, x)] >= 0) continue;
        const uint32_t g = sig[at(z, y, x)];
        int64_t wx = 1, wy = 1, wz = 1;
        while (wx < M && x + wx < nb2 && free_same(z, y, x + wx, g)) wx++;
        for (bool grow = true; grow && wy < M && y + wy < nb1;) {
          for (int64_t i = 0; i < wx && grow; i++) grow = free_same(z, y + wy, x + i, g);
          if (grow) wy++;
        }
        for (bool grow = true; grow && wz < M && z + wz < nb0;) {
          for (int64_t j = 0; j < wy && grow; j++)
            for (int64_t i = 0; i < wx && grow; i++) grow = free_same(z + wz, y + j, x + i, g);
          if (grow) wz++;
        }
        const int32_t id = (int32_t)(box.size() / 8);
        for (int64_t k = 0; k < wz; k++)
          for (int64_t j = 0; j < wy; j++)
            for (int64_t i = 0; i < wx; i++) unit[at(z + k, y + j, x + i)] = id;
        const uint32_t e[8] = {(uint32_t)z, (uint32_t)y, (uint32_t)x, (uint32_t)(z + wz), (uint32_t)(y + wy),
                               (uint32_t)(x + wx), 0u, 0u};
        box.insert(box.end(), e, e + 8);
      }
  const int64_t U = (int64_t)(box.size() / 8);
  // slots of every (unit, level) in order, the largest unit
  std::vector<int64_t> ubase((size_t)(U * gb.nL));
  uint32_t maxch[kMaxLevels] = {};
  int mb[3] = {1, 1, 1};
  int64_t base = 0;
  for (int64_t u = 0; u < U; u++) {
    int64_t o[3], hi[3];
    for (int a = 0; a < 3; a++) {
      o[a] = (int64_t)box[8 * u + a] * gb.B;
      hi[a] = std::min<int64_t>((int64_t)box[8 * u + 3 + a] * gb.B, gb.n[a] - 1);
      mb[a] = std::max<int>(mb[a], (int)(box[8 * u + 3 + a] - box[8 * u + a]));
    }
    for (int l = L; l >= 0; l--) {
      const uint32_t nch = (uint32_t)((sec_geom(o, hi, l, L).npts + 63) / 64);
      ubase[(size_t)(u * gb.nL + (L - l))] = base;
      base += nch;
      maxch[l] = std::max(maxch[l], nch);
    }
  }
  if (hipMemcpyAsync(J.units, box.data(), sizeof(uint32_t) * box.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(J.ubase, ubase.data(), sizeof(int64_t) * ubase.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(CHR_E_HIP, "merged units: copy to the device failed");
  // the plan over units (every size here is within the workspace layout's
  // bounds for merged units)
  P.g.units = J.units;
  P.g.nblocks = U;
  for (int a = 0; a < 3; a++) P.g.mb[a] = mb[a];
  P.ubase = J.ubase;
  P.nslots = base;
  for (int l = 0; l < kMaxLevels; l++) P.maxch[l] = l <= L ? maxch[l] : 0;
  P.part_l1 = encode_fine_groups(P);
  P.part_l2 = P.part_l1 + encode_l1_groups(P);
  P.part_per_block = P.part_l2 + encode_l2_groups(P) + 1;
  encode_pack_layout(P);
  P.payload_off = kHeaderBytes + (uint64_t)U * (16 * (uint64_t)gb.nL + 16 + 32);
  if (P.cap < P.payload_off) return fail(CHR_E_CAPACITY, "capacity below the header and tables");
  return CHR_OK;
}

// Workspace of a reconstruction to `level`: the compact grids of the levels
// above it (the output holds level `level` itself).
static size_t dec_need(const Geo &g, int level) {
  const int L = g.nL - 1;
  size_t need = 0;
  for (int l = std::max(level, 1); l <= L; l++) {
    if (l == level) continue;
    need = align256(need + sizeof(float) * (size_t)(lvl_dim(g.n[0], l) * lvl_dim(g.n[1], l) * lvl_dim(g.n[2], l)));
  }
  return need;
}

size_t dec_workspace_bytes(const Geo &g, int level) { return std::max<size_t>(dec_need(g, level), 256); }

int dec_prepare(const Geo &g, uint64_t payload_off, int level, const void *d_stream, uint64_t stream_bytes,
                float *d_out, int32_t *d_status, void *d_ws, size_t ws_bytes, int cpw0, DecJob &J) {
  DecPlan &D = J.D;
  std::memset(&D, 0, sizeof(D));
  if (!d_stream || !d_out) return fail(CHR_E_INVAL, "NULL argument");
  if (reinterpret_cast<uintptr_t>(d_stream) & 7) return fail(CHR_E_INVAL, "stream must be 8-byte aligned");
  if (level < 0 || level >= g.nL) return fail(CHR_E_LEVEL, "level outside the hierarchy");
  if (g.nblocks > 65535) return fail(CHR_E_INVAL, "more than 65535 blocks");
  const size_t need = dec_need(g, level);
  if (ws_bytes < need || (need && !d_ws)) return fail(CHR_E_NOMEM, "workspace too small: need " + std::to_string(need));
  D.g = g;
  make_l0geo(D.g, D.l0);
  if (g.merge > 1) {
    // merged units: their boxes from the stream's box table, general kernels
    D.g.units = reinterpret_cast<const uint32_t *>(static_cast<const uint8_t *>(d_stream) + payload_off -
                                                  32 * (uint64_t)g.nblocks);
    D.l0.small = 0;
  }
  D.cpw0 = cpw0;
  D.tile0 = g_tune.tile0;
  D.lo = level;
  const int L = g.nL - 1;
  for (int l = 0; l < kMaxLevels; l++)
    for (int a = 0; a < 3; a++) D.gd[l][a] = (l <= L) ? lvl_dim(g.n[a], l) : 0;
  size_t off = 0;
  uint8_t *ws = static_cast<uint8_t *>(d_ws);
  for (int l = std::max(level, 1); l <= L; l++) {
    if (l == level) { D.gp[l] = d_out; continue; }
    D.gp[l] = reinterpret_cast<float *>(ws + off);
    off = align256(off + sizeof(float) * (size_t)(D.gd[l][0] * D.gd[l][1] * D.gd[l][2]));
  }
  D.payload_off = payload_off;
  D.s = static_cast<const uint8_t *>(d_stream);
  D.sbytes = stream_bytes;
  D.out = d_out;
  D.status = d_status;
  return CHR_OK;
}

static int mc_plan(const float *d_field, const int64_t dims[3], McPlan &M, size_t &need, size_t off[7]) {
  std::memset(&M, 0, sizeof(M));
  if (!dims_ok(dims)) return fail(CHR_E_INVAL, "dims must be in [1, 2^30]");
  for (int a = 0; a < 3; a++) M.n[a] = dims[a];
  M.nrows = dims[0] * dims[1];
  M.nw = ceil_div(dims[2], 64);
  if ((double)M.nrows * (double)M.nw * 64.0 >= 4294967296.0)
    return fail(CHR_E_INVAL, "field too large for marching cubes (2^32 padded points)");
  M.f = d_field;
  M.py = dims[2];
  M.pz = dims[1] * dims[2];
  size_t o = 0;
  off[0] = o; o = align256(o + 8 * (size_t)(M.nrows * M.nw));
  const int64_t nwords = M.nrows * M.nw;
  off[1] = o; o = align256(o + sizeof(uint32_t) * (size_t)nwords);
  off[2] = o; o = align256(o + sizeof(U4) * (size_t)(nwords + 1));
  off[3] = o; o = align256(o + sizeof(U4) * (size_t)scan_tmp_elems(nwords));
  off[4] = o; o = align256(o + sizeof(uint32_t) * (size_t)(nwords * 64));
  off[5] = o; o = align256(o + sizeof(uint32_t) * (size_t)(nwords * 64));
  off[6] = o; o = align256(o + sizeof(uint32_t) * (size_t)(nwords / 4 + 1));
  need = o;
  return CHR_OK;
}

size_t mc_workspace_bytes(const int64_t dims[3]) {
  McPlan M;
  size_t need = 0, off[7];
  if (mc_plan(nullptr, dims, M, need, off)) return 0;
  return need;
}

int mc_prepare(const float *d_field, const int64_t dims[3], float isovalue, float spacing, float *d_vertices,
               int64_t cap_v, int32_t *d_tris, int64_t cap_t, int64_t *d_counts, void *d_ws, size_t ws_bytes,
               McJob &J) {
  if (!d_field || !d_counts || !d_ws) return fail(CHR_E_INVAL, "NULL argument");
  if (cap_v < 0 || cap_t < 0 || (cap_v && !d_vertices) || (cap_t && !d_tris)) return fail(CHR_E_INVAL, "bad capacity");
  if (!std::isfinite(isovalue) || !std::isfinite(spacing)) return fail(CHR_E_INVAL, "isovalue and spacing must be finite");
  McPlan &M = J.M;
  size_t need = 0, off[7];
  int rc = mc_plan(d_field, dims, M, need, off);
  if (rc) return rc;
  if (ws_bytes < need) return fail(CHR_E_NOMEM, "workspace too small: need " + std::to_string(need));
  uint8_t *ws = static_cast<uint8_t *>(d_ws);
  M.bits = reinterpret_cast<unsigned long long *>(ws + off[0]);
  M.cnt = reinterpret_cast<uint32_t *>(ws + off[1]);
  M.P = reinterpret_cast<U4 *>(ws + off[2]);
  M.vlist = reinterpret_cast<uint32_t *>(ws + off[4]);
  M.clist = reinterpret_cast<uint32_t *>(ws + off[5]);
  M.tb = reinterpret_cast<uint32_t *>(ws + off[6]);
  M.cap_pv = M.cap_ac = M.nrows * M.nw * 64;
  M.k = isovalue;
  M.spacing = spacing;
  M.verts = d_vertices;
  M.tris = d_tris;
  M.cap_v = cap_v;
  M.cap_t = cap_t;
  M.counts = d_counts;
  J.scan = reinterpret_cast<U4 *>(ws + off[3]);
  return CHR_OK;
}

// Geometry of a stream from its parsed header, checked for consistency.
int info_geo(const chr_info *I, Geo &g) {
  const bool merged = (I->flags & 8u) != 0;
  chr_params p{I->levels, I->block, I->qmax, 0.0, merged ? I->merge : 0};
  std::string why;
  if (!params_ok(I->dims, &p, why)) return fail(CHR_E_CORRUPT, why);
  fill_geo(g, I->dims, I->levels, I->block, I->qmax);
  if (merged) {
    // storage units: the merged units (their boxes are read on the device)
    if (I->merge < 2 || I->nblocks < 1 || I->nblocks > g.nblocks) return fail(CHR_E_CORRUPT, "bad merged units");
    set_merge(g, I->merge);
    g.nblocks = I->nblocks;
    for (int a = 0; a < 3; a++) {
      if (I->mb[a] < 1 || I->mb[a] > I->merge) return fail(CHR_E_CORRUPT, "bad largest unit");
      g.mb[a] = I->mb[a];
    }
  }
  set_quant(g, I->error_bound);
  if (std::memcmp(&g.inv, &I->inv, 4) || std::memcmp(&g.step, &I->step, 4))
    return fail(CHR_E_CORRUPT, "quantizer constants do not match the error bound");
  if ((g.lossless ? 1u : 0u) != (I->flags & 1u)) return fail(CHR_E_CORRUPT, "lossless flag mismatch");
  if (I->flags & 2u) {
    if (!(I->error_bound_far >= I->error_bound && std::isfinite(I->error_bound_far)))
      return fail(CHR_E_CORRUPT, "bad far error bound");
    set_quant_far(g, I->error_bound_far);
    if (std::memcmp(&g.inv2, &I->inv_far, 4) || std::memcmp(&g.step2, &I->step_far, 4))
      return fail(CHR_E_CORRUPT, "far quantizer constants do not match the far error bound");
    if ((g.lossless2 ? 4u : 0u) != (I->flags & 4u)) return fail(CHR_E_CORRUPT, "far lossless flag mismatch");
  }
  if (I->n_iso < 0 || I->n_iso > kMaxIso) return fail(CHR_E_CORRUPT, "bad isovalue count");
  g.K = I->n_iso;
  for (int j = 0; j < kMaxIso; j++) g.iso[j] = I->isovalues[j];
  return CHR_OK;
}

void prof_mark(const char *kernel, hipStream_t s, int end) {
  if (!g_prof.on || g_prof.name != kernel) return;
  if (!end && g_prof.used + 2 > (int)g_prof.ev.size()) return;
  if (end && (g_prof.used & 1) == 0) return;  // its begin was not recorded
  hipEventRecord(g_prof.ev[g_prof.used], s);
  g_prof.used++;
}
}  // namespace chr

extern "C" {

int chr_prof_enable(const char *kernel, int max_launches) {
  if (!kernel || max_launches < 1) return fail(CHR_E_INVAL, "bad argument");
  chr_prof_disable();
  g_prof.ev.resize(2 * (size_t)max_launches);
  for (auto &e : g_prof.ev)
    if (hipEventCreate(&e) != hipSuccess) return fail(CHR_E_HIP, "hipEventCreate failed");
  g_prof.name = kernel;
  g_prof.used = 0;
  g_prof.on = true;
  return CHR_OK;
}

int chr_prof_collect(float *ms, int max, int *n_out) {
  if (!n_out) return fail(CHR_E_INVAL, "bad argument");
  int n = 0;
  for (int i = 0; i + 1 < g_prof.used && n < max; i += 2) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, g_prof.ev[i], g_prof.ev[i + 1]) != hipSuccess) return fail(CHR_E_HIP, "event timing failed");
    if (ms) ms[n] = t;
    n++;
  }
  *n_out = n;
  g_prof.used = 0;
  return CHR_OK;
}

int chr_prof_disable(void) {
  for (auto &e : g_prof.ev) hipEventDestroy(e);
  g_prof.ev.clear();
  g_prof.used = 0;
  g_prof.on = false;
  return CHR_OK;
}

const char *chr_last_error(void) { return g_err.c_str(); }

int chr_set_tiles(int enc_chunks_per_wave, int dec_chunks_per_wave) {
  if (!tiles_ok(enc_chunks_per_wave, dec_chunks_per_wave))
    return fail(CHR_E_INVAL, "tiles: compression 1, 2, 4, 8 or 16; reconstruction 8, 16, 32 or 64 chunks per wave");
  g_tune.enc_cpw0 = enc_chunks_per_wave;
  g_tune.dec_cpw0 = dec_chunks_per_wave;
  return CHR_OK;
}

int chr_set_level0_tiles(int on) {
  if (on != 0 && on != 1) return fail(CHR_E_INVAL, "chr_set_level0_tiles: 0 or 1");
  g_tune.tile0 = on;
  return CHR_OK;
}

int chr_version(void) { return 1; }

size_t chr_compress_bound(const int64_t dims[3], const chr_params *p) {
  std::string why;
  if (!params_ok(dims, p, why)) { g_err = why; return 0; }
  Geo g;
  fill_geo(g, dims, p->levels, p->block, p->qmax);
  const int L = g.nL - 1;
  size_t total = kHeaderBytes + 16 * (size_t)g.nblocks * g.nL + 16 * (size_t)g.nblocks;
  // merged units: no larger than their blocks' sections, plus a box entry each
  if (p->merge > 1) total += 32 * (size_t)g.nblocks;
  AxisClass ac[3];
  for (int a = 0; a < 3; a++) ac[a] = axis_classes(dims[a], p->block);
  for (int iz = 0; iz < ac[0].n; iz++)
    for (int iy = 0; iy < ac[1].n; iy++)
      for (int ix = 0; ix < ac[2].n; ix++) {
        int64_t o[3] = {0, 0, 0}, hi[3] = {ac[0].ext[iz], ac[1].ext[iy], ac[2].ext[ix]};
        int64_t cnt = ac[0].count[iz] * ac[1].count[iy] * ac[2].count[ix];
        for (int l = L; l >= 0; l--) {
          Sec s = sec_geom(o, hi, l, L);
          uint64_t nch = (s.npts + 63) / 64;
          total += (size_t)cnt * sec_bytes(s.npts, 16 * nch, nch, s.npts);
        }
      }
  return total;
}

size_t chr_compress_workspace(const int64_t dims[3], const chr_params *p) { return enc_workspace_bytes(dims, p); }

int chr_compress(const float *d_field, const int64_t dims[3], double error_bound, const float *h_isovalues,
                 int n_iso, const chr_params *p, void *d_stream, size_t capacity, chr_result *d_result,
                 int32_t *d_codes, uint8_t *d_flags, void *d_ws, size_t ws_bytes, void *stream) {
  EncJob J;
  int rc = enc_prepare(d_field, dims, error_bound, h_isovalues, n_iso, p, d_stream, capacity, d_result, d_codes,
                       d_flags, d_ws, ws_bytes, g_tune.enc_cpw0, J, true);
  if (rc) return rc;
  if (J.P.g.merge > 1) {
    rc = enc_merge_units(J, static_cast<hipStream_t>(stream));
    if (rc) return rc;
  }
  launch_encode(J.P, 0, J.scan, J.scan64, static_cast<hipStream_t>(stream));
  return check_hip("chr_compress launch");
}

int chr_stream_info(const void *h_stream, size_t n, chr_info *I) {
  if (!h_stream || !I) return fail(CHR_E_INVAL, "NULL argument");
  const uint8_t *s = static_cast<const uint8_t *>(h_stream);
  if (n < (size_t)kHeaderBytes) return fail(CHR_E_CORRUPT, "stream shorter than its header");
  if (rd<uint32_t>(s) != kMagic || rd<uint32_t>(s + 4) != kVersion) return fail(CHR_E_CORRUPT, "bad magic or version");
  if (host_checksum(s, 252) != rd<uint32_t>(s + 252)) return fail(CHR_E_CORRUPT, "header checksum mismatch");
  std::memset(I, 0, sizeof(*I));
  for (int a = 0; a < 3; a++) I->dims[a] = rd<int64_t>(s + 8 + 8 * a);
  I->levels = rd<int32_t>(s + 32);
  I->block = rd<int32_t>(s + 36);
  I->qmax = rd<int32_t>(s + 40);
  I->n_iso = rd<int32_t>(s + 44);
  I->error_bound = rd<double>(s + 48);
  I->inv = rd<float>(s + 56);
  I->step = rd<float>(s + 60);
  for (int j = 0; j < kMaxIso; j++) I->isovalues[j] = rd<float>(s + 64 + 4 * j);
  I->vmin = rd<float>(s + 128);
  I->vmax = rd<float>(s + 132);
  I->nblocks = rd<int64_t>(s + 136);
  for (int a = 0; a < 3; a++) I->nb[a] = rd<int32_t>(s + 144 + 4 * a);
  I->flags = rd<uint32_t>(s + 156);
  I->total_bytes = rd<uint64_t>(s + 160);
  I->n_outlier = rd<uint64_t>(s + 168);
  I->n_corrected = rd<uint64_t>(s + 176);
  I->payload_offset = rd<uint64_t>(s + 184);
  I->error_bound_far = rd<double>(s + 192);
  I->inv_far = rd<float>(s + 200);
  I->step_far = rd<float>(s + 204);
  const bool merged = (I->flags & 8u) != 0;
  I->merge = merged ? rd<int32_t>(s + 208) : 1;
  for (int a = 0; a < 3; a++) I->mb[a] = merged ? rd<int32_t>(s + 212 + 4 * a) : 1;
  if (I->flags & ~15u) return fail(CHR_E_CORRUPT, "unknown flags");
  if (merged && (I->flags & 2u)) return fail(CHR_E_CORRUPT, "merged units with differentiated bounds");
  chr_params p{I->levels, I->block, I->qmax, 0.0, merged ? I->merge : 0};
  std::string why;
  if (!params_ok(I->dims, &p, why)) return fail(CHR_E_CORRUPT, "header parameters invalid: " + why);
  if (merged && I->merge < 2) return fail(CHR_E_CORRUPT, "bad merge");
  if (I->n_iso < 0 || I->n_iso > kMaxIso) return fail(CHR_E_CORRUPT, "bad isovalue count");
  Geo g;
  fill_geo(g, I->dims, I->levels, I->block, I->qmax);
  if (g.nb[0] != I->nb[0] || g.nb[1] != I->nb[1] || g.nb[2] != I->nb[2]) return fail(CHR_E_CORRUPT, "block grid mismatch");
  if (merged ? (I->nblocks < 1 || I->nblocks > g.nblocks) : g.nblocks != I->nblocks)
    return fail(CHR_E_CORRUPT, "unit count mismatch");
  for (int a = 0; a < 3; a++)
    if (I->mb[a] < 1 || I->mb[a] > I->merge) return fail(CHR_E_CORRUPT, "bad largest unit");
  if (I->payload_offset != kHeaderBytes + 16 * (uint64_t)I->nblocks * I->levels + 16 * (uint64_t)I->nblocks +
                               (merged ? 32 * (uint64_t)I->nblocks : 0))
    return fail(CHR_E_CORRUPT, "payload offset mismatch");
  if (I->payload_offset > I->total_bytes) return fail(CHR_E_CORRUPT, "total size below the tables");
  if (n >= I->payload_offset) {
    if (host_checksum(s + kHeaderBytes, I->payload_offset - kHeaderBytes) != rd<uint32_t>(s + 248))
      return fail(CHR_E_CORRUPT, "table checksum mismatch");
    if (merged) {
      // the units tile the block grid, none wider than the largest stated
      std::vector<uint8_t> seen((size_t)g.nblocks, 0);
      const uint8_t *xt = s + I->payload_offset - 32 * (size_t)I->nblocks;
      for (int64_t u = 0; u < I->nblocks; u++) {
        uint32_t e[8];
        std::memcpy(e, xt + 32 * (size_t)u, 32);
        if (e[6] || e[7]) return fail(CHR_E_CORRUPT, "bad box entry");
        for (int a = 0; a < 3; a++)
          if (e[a] >= e[3 + a] || e[3 + a] > (uint32_t)g.nb[a] || e[3 + a] - e[a] > (uint32_t)I->mb[a])
            return fail(CHR_E_CORRUPT, "bad box entry");
        for (uint32_t z = e[0]; z < e[3]; z++)
          for (uint32_t y = e[1]; y < e[4]; y++)
            for (uint32_t x = e[2]; x < e[5]; x++) {
              uint8_t &f = seen[(size_t)(((int64_t)z * g.nb[1] + y) * g.nb[2] + x)];
              if (f) return fail(CHR_E_CORRUPT, "overlapping units");
              f = 1;
            }
      }
      for (uint8_t f : seen)
        if (!f) return fail(CHR_E_CORRUPT, "units leave a block out");
    }
  }
  return CHR_OK;
}

int chr_stream_verify(const void *h_stream, size_t n) {
  chr_info I;
  int rc = chr_stream_info(h_stream, n, &I);
  if (rc) return rc;
  if (n < I.total_bytes) return fail(CHR_E_CORRUPT, "stream truncated");
  if (n < I.payload_offset) return fail(CHR_E_CORRUPT, "stream truncated");
  const uint8_t *s = static_cast<const uint8_t *>(h_stream);
  const size_t btab = kHeaderBytes + 16 * (size_t)I.nblocks * I.levels;
  for (int64_t b = 0; b < I.nblocks; b++) {
    const uint8_t *first = s + kHeaderBytes + 16 * (size_t)b * I.levels;
    const uint8_t *last = s + kHeaderBytes + 16 * ((size_t)b * I.levels + I.levels - 1);
    uint64_t start = rd<uint64_t>(first), end = rd<uint64_t>(last) + rd<uint64_t>(last + 8);
    if (start > end || end > I.total_bytes) return fail(CHR_E_CORRUPT, "section table out of range");
    if (host_checksum(s + start, end - start) != rd<uint32_t>(s + btab + 16 * (size_t)b + 8))
      return fail(CHR_E_CORRUPT, "block checksum mismatch");
  }
  return CHR_OK;
}

size_t chr_reconstruct_workspace(const chr_info *info, int level) {
  if (!info) return 0;
  Geo g;
  if (info_geo(info, g)) return 0;
  if (level < 0 || level >= g.nL) { g_err = "level outside the hierarchy"; return 0; }
  return dec_workspace_bytes(g, level);
}

int chr_reconstruct(const chr_info *info, const void *d_stream, size_t stream_bytes, int level, double error_bound,
                    float *d_out, int32_t *d_status, void *d_ws, size_t ws_bytes, void *stream) {
  return chr::reconstruct_impl(info, d_stream, stream_bytes, level, error_bound, nullptr, d_out, d_status, d_ws,
                               ws_bytes, stream);
}

int chr_reconstruct_range(const chr_info *info, const void *d_stream, size_t stream_bytes, int level,
                          double error_bound, float kmin, float kmax, float *d_out, int32_t *d_status, void *d_ws,
                          size_t ws_bytes, void *stream) {
  if (!std::isfinite(kmin) || !std::isfinite(kmax) || !(kmin <= kmax))
    return fail(CHR_E_INVAL, "isovalue range must be finite with kmin <= kmax");
  const float kr[2] = {kmin, kmax};
  return chr::reconstruct_impl(info, d_stream, stream_bytes, level, error_bound, kr, d_out, d_status, d_ws, ws_bytes,
                               stream);
}

}  // extern "C"

namespace chr {

size_t reconstruct_need(const chr_info *info, int level) {
  Geo g;
  if (!info || info_geo(info, g) || level < 0 || level >= g.nL) return 0;
  return dec_need(g, level);
}

int reconstruct_impl(const chr_info *info, const void *d_stream, size_t stream_bytes, int level, double error_bound,
                     const float *krange, float *d_out, int32_t *d_status, void *d_ws, size_t ws_bytes,
                     void *stream) {
  if (!info || !d_stream || !d_out) return fail(CHR_E_INVAL, "NULL argument");
  Geo g;
  int rc = info_geo(info, g);
  if (rc) return rc;
  if (level < 0 || level >= g.nL) return fail(CHR_E_LEVEL, "level outside the hierarchy");
  if (!(error_bound >= stream_bound(*info))) return fail(CHR_E_ACCURACY, "requested error bound below the stream's");
  if (stream_bytes < info->total_bytes) return fail(CHR_E_CORRUPT, "stream shorter than its header states");
  DecJob J;
  rc = dec_prepare(g, info->payload_offset, level, d_stream, info->total_bytes, d_out, d_status, d_ws, ws_bytes,
                   g_tune.dec_cpw0, J);
  if (rc) return rc;
  if (krange) {
    J.D.prune = 1;
    J.D.kmin = krange[0];
    J.D.kmax = krange[1];
  }
  launch_decode(J.D, static_cast<hipStream_t>(stream));
  return check_hip("chr_reconstruct launch");
}

}  // namespace chr

extern "C" {

size_t iso_workspace(const int64_t dims[3]) { return mc_workspace_bytes(dims); }

int iso_extract_bits(const float *d_field, const int64_t dims[3], const uint64_t *d_bits, float isovalue,
                     float spacing, float *d_vertices, int64_t cap_v, int32_t *d_tris, int64_t cap_t,
                     int64_t *d_counts, void *d_ws, size_t ws_bytes, void *stream) {
  if (!d_bits) return fail(CHR_E_INVAL, "NULL bits");
  McJob J;
  int rc = mc_prepare(d_field, dims, isovalue, spacing, d_vertices, cap_v, d_tris, cap_t, d_counts, d_ws, ws_bytes, J);
  if (rc) return rc;
  J.M.bits = const_cast<unsigned long long *>(reinterpret_cast<const unsigned long long *>(d_bits));
  launch_mc_from_bits(J.M, J.scan, static_cast<hipStream_t>(stream));
  return check_hip("iso_extract_bits launch");
}

int chr_reconstruct_bits(const chr_info *info, const void *d_stream, size_t stream_bytes, double error_bound,
                         const float *h_isovalues, int n_iso, float *d_out, uint64_t *d_bits, int32_t *d_status,
                         void *d_ws, size_t ws_bytes, void *stream) {
  if (!info || !d_stream || !d_out || !d_bits || !h_isovalues) return fail(CHR_E_INVAL, "NULL argument");
  if (n_iso < 1 || n_iso > kMaxIso) return fail(CHR_E_INVAL, "n_iso must be in [1, 16]");
  for (int j = 0; j < n_iso; j++)
    if (!std::isfinite(h_isovalues[j])) return fail(CHR_E_INVAL, "isovalues must be finite");
  Geo g;
  int rc = info_geo(info, g);
  if (rc) return rc;
  if (!(error_bound >= stream_bound(*info))) return fail(CHR_E_ACCURACY, "requested error bound below the stream's");
  if (stream_bytes < info->total_bytes) return fail(CHR_E_CORRUPT, "stream shorter than its header states");
  McPlan M;
  size_t mneed = 0, moff[7];
  rc = mc_plan(d_out, info->dims, M, mneed, moff);
  if (rc) return rc;
  DecJob J;
  rc = dec_prepare(g, info->payload_offset, 0, d_stream, info->total_bytes, d_out, d_status, d_ws, ws_bytes,
                   g_tune.dec_cpw0, J);
  if (rc) return rc;
  DecPlan &D = J.D;
  D.bits = reinterpret_cast<unsigned long long *>(d_bits);
  D.bnw = M.nw;
  D.bplane = M.nrows * M.nw;
  D.nk = n_iso;
  for (int j = 0; j < n_iso; j++) D.kb[j] = h_isovalues[j];
  hipStream_t s = static_cast<hipStream_t>(stream);
  launch_decode(D, s);
  if (!decode_tile0_used(D)) {
    // another decoder ran: one classification pass per isovalue
    for (int j = 0; j < n_iso; j++) {
      M.bits = D.bits + (size_t)j * (size_t)D.bplane;
      M.k = h_isovalues[j];
      launch_mc_bits(M, s);
    }
  }
  return check_hip("chr_reconstruct_bits launch");
}

int iso_extract(const float *d_field, const int64_t dims[3], float isovalue, float spacing, float *d_vertices,
                int64_t cap_v, int32_t *d_tris, int64_t cap_t, int64_t *d_counts, void *d_ws, size_t ws_bytes,
                void *stream) {
  McJob J;
  int rc = mc_prepare(d_field, dims, isovalue, spacing, d_vertices, cap_v, d_tris, cap_t, d_counts, d_ws, ws_bytes, J);
  if (rc) return rc;
  launch_mc(J.M, J.scan, static_cast<hipStream_t>(stream));
  return check_hip("iso_extract launch");
}

int chr_block_box(const void *h_head, size_t head_bytes, float kmin, float kmax, int64_t lo[3], int64_t hi[3],
                  int *found) {
  if (!h_head || !lo || !hi || !found) return fail(CHR_E_INVAL, "NULL argument");
  if (!std::isfinite(kmin) || !std::isfinite(kmax) || !(kmin <= kmax))
    return fail(CHR_E_INVAL, "isovalue range must be finite with kmin <= kmax");
  chr_info I;
  int rc = chr_stream_info(h_head, head_bytes, &I);
  if (rc) return rc;
  if (head_bytes < I.payload_offset) return fail(CHR_E_INVAL, "h_head must hold the header and tables");
  Geo g;
  rc = info_geo(&I, g);
  if (rc) return rc;
  const uint8_t *s = static_cast<const uint8_t *>(h_head);
  const size_t btab = kHeaderBytes + 16 * (size_t)I.nblocks * I.levels;
  int64_t blo[3] = {INT64_MAX, INT64_MAX, INT64_MAX}, bhi[3] = {-1, -1, -1};
  int any = 0;
  for (int64_t b = 0; b < I.nblocks; b++) {
    const float mn = rd<float>(s + btab + 16 * (size_t)b), mx = rd<float>(s + btab + 16 * (size_t)b + 4);
    if (!(mn < mx && mn < kmax && kmin <= mx)) continue;
    int64_t o[3], h[3];
    if (g.merge > 1) {
      uint32_t e[8];
      std::memcpy(e, s + I.payload_offset - 32 * (size_t)I.nblocks + 32 * (size_t)b, 32);
      for (int a = 0; a < 3; a++) {
        o[a] = (int64_t)e[a] * g.B;
        h[a] = std::min<int64_t>((int64_t)e[3 + a] * g.B, g.n[a] - 1);
      }
    } else {
      block_ext(g, b, o, h);
    }
    for (int a = 0; a < 3; a++) {
      blo[a] = std::min(blo[a], o[a]);
      bhi[a] = std::max(bhi[a], h[a]);
    }
    any = 1;
  }
  *found = any;
  if (any)
    for (int a = 0; a < 3; a++) { lo[a] = blo[a]; hi[a] = bhi[a]; }
  return CHR_OK;
}

size_t iso_box_workspace(const int64_t box_dims[3]) { return mc_workspace_bytes(box_dims); }

int iso_extract_box(const float *d_field, const int64_t dims[3], const int64_t lo[3], const int64_t hi[3],
                    float isovalue, float spacing, float *d_vertices, int64_t cap_v, int32_t *d_tris, int64_t cap_t,
                    int64_t *d_counts, void *d_ws, size_t ws_bytes, void *stream) {
  if (!d_field || !dims || !lo || !hi || !d_ws) return fail(CHR_E_INVAL, "NULL argument");
  if (!dims_ok(dims)) return fail(CHR_E_INVAL, "dims must be in [1, 2^30]");
  int64_t bd[3];
  for (int a = 0; a < 3; a++) {
    if (lo[a] < 0 || hi[a] >= dims[a] || lo[a] > hi[a]) return fail(CHR_E_INVAL, "box outside the field or empty");
    bd[a] = hi[a] - lo[a] + 1;
  }
  const size_t need = iso_box_workspace(bd);
  if (need == 0) return fail(CHR_E_INVAL, "box too large");
  if (ws_bytes < need) return fail(CHR_E_NOMEM, "workspace too small: need " + std::to_string(need));
  // the box read in place: its first point, the field's row and plane pitches
  const float *f0 = d_field + (lo[0] * dims[1] + lo[1]) * dims[2] + lo[2];
  McJob J;
  int rc = mc_prepare(f0, bd, isovalue, spacing, d_vertices, cap_v, d_tris, cap_t, d_counts, d_ws, ws_bytes, J);
  if (rc) return rc;
  for (int a = 0; a < 3; a++) J.M.org[a] = (uint32_t)lo[a];
  J.M.py = dims[2];
  J.M.pz = dims[1] * dims[2];
  launch_mc(J.M, J.scan, static_cast<hipStream_t>(stream));
  return check_hip("iso_extract_box launch");
}

int iso_cases(const float *d_field, const int64_t dims[3], float isovalue, uint8_t *d_cases, void *d_ws,
              size_t ws_bytes, void *stream) {
  if (!d_field || !d_cases || !d_ws) return fail(CHR_E_INVAL, "NULL argument");
  McPlan M;
  size_t need = 0, off[7];
  int rc = mc_plan(d_field, dims, M, need, off);
  if (rc) return rc;
  if (ws_bytes < need) return fail(CHR_E_NOMEM, "workspace too small");
  uint8_t *ws = static_cast<uint8_t *>(d_ws);
  M.bits = reinterpret_cast<unsigned long long *>(ws + off[0]);
  M.k = isovalue;
  M.cases = d_cases;
  launch_mc_cases(M, static_cast<hipStream_t>(stream));
  return check_hip("iso_cases launch");
}

int chr_mc_table(uint8_t *ntri, int8_t *tri) {
  if (!ntri || !tri) return fail(CHR_E_INVAL, "NULL argument");
  mc_table_host(ntri, tri);
  return CHR_OK;
}

size_t chr_topology_workspace(void) { return align256(topo_workspace_bytes()); }

int chr_topology_error_bound(const float *d_field, const int64_t dims[3], const float *h_isovalues, int n_iso,
                             int64_t nth, double *d_out, void *d_ws, size_t ws_bytes, void *stream) {
  if (!d_field || !d_out || !d_ws) return fail(CHR_E_INVAL, "NULL argument");
  if (!dims_ok(dims)) return fail(CHR_E_INVAL, "dims must be in [1, 2^30]");
  if ((double)dims[0] * (double)dims[1] * (double)ceil_div(dims[2], 64) >= 2147483648.0)
    return fail(CHR_E_INVAL, "more than 2^31 words of 64 points");
  if (n_iso < 0 || n_iso > kMaxIso || (n_iso > 0 && !h_isovalues)) return fail(CHR_E_INVAL, "n_iso must be in [0, 16]");
  for (int j = 0; j < n_iso; j++)
    if (!std::isfinite(h_isovalues[j])) return fail(CHR_E_INVAL, "isovalues must be finite");
  if (ws_bytes < align256(topo_workspace_bytes())) return fail(CHR_E_NOMEM, "workspace too small");
  launch_topology(d_field, dims, h_isovalues, n_iso, nth, d_out, d_ws, static_cast<hipStream_t>(stream));
  return check_hip("chr_topology_error_bound launch");
}

int chr_range(const float *d_field, int64_t n, float *d_out, void *stream) {
  if (!d_field || !d_out || n < 1) return fail(CHR_E_INVAL, "bad argument");
  launch_range(d_field, n, d_out, static_cast<hipStream_t>(stream));
  return check_hip("chr_range launch");
}

}  // extern "C"
