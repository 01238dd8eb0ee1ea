// decode.hip -- CHR reconstruction kernels for gfx950 (the visualization
// side's reconstruction of the requested level, Sec. II).
//
// One 64-lane wave decodes one tile (64 chunks = 4096 points) of a section:
// lane t reads chunk t's header byte, wave prefix sums over the widths and
// exact flags (plus the tile's stored base offsets) locate every chunk's
// codes, exact mask and exact values; then for each chunk every lane unpacks
// its w-bit code with one or two aligned 32-bit loads, predicts its point
// exactly as compression did, and writes x' = exact value or p + q*2e.
// Coarse levels run one workgroup per block (levels nL-1 .. max(lo,1)); level
// 0 runs over (tile groups, blocks) and writes whole output rows, taking the
// even points of even rows from the level-1 grid.
#include "chr_plan.h"

namespace chr {
namespace {

constexpr int kBS = 256;
constexpr int kWaves = kBS / kWave;
constexpr int kDecGroup = 2;  // level-0 decoder: chunks whose loads a wave issues together

// Same prediction as compression (multilinear midpoints from the coarser
// compact grid of dims g0 x g1 x g2, x then y then z, lower parent alone at
// the domain edge).
__device__ inline float predict(const float *__restrict__ Gp, uint32_t g0, uint32_t g1, uint32_t g2, int l,
                                uint32_t z, uint32_t y, uint32_t x) {
  const int sh = l + 1;
  const uint32_t oz = (z >> l) & 1u, oy = (y >> l) & 1u, ox = (x >> l) & 1u;
  const uint32_t zl = (z - (oz << l)) >> sh;
  const uint32_t yl = (y - (oy << l)) >> sh;
  const uint32_t xl = (x - (ox << l)) >> sh;
  const bool zu = oz && (zl + 1 < g0);
  const bool yu = oy && (yl + 1 < g1);
  const bool xu = ox && (xl + 1 < g2);
  const uint32_t zb = zu ? zl + 1 : zl, yb = yu ? yl + 1 : yl, xb = xu ? xl + 1 : xl;
  const float *r00 = Gp + ((size_t)zl * g1 + yl) * g2, *r01 = Gp + ((size_t)zl * g1 + yb) * g2;
  const float *r10 = Gp + ((size_t)zb * g1 + yl) * g2, *r11 = Gp + ((size_t)zb * g1 + yb) * g2;
  return midpoint_rows(r00, r01, r10, r11, xl, xb, zu, yu, xu);
}

__device__ inline uint32_t ld32(const uint8_t *p) { return *reinterpret_cast<const uint32_t *>(p); }
__device__ inline uint64_t ld64(const uint8_t *p) {
  const uint32_t *q = reinterpret_cast<const uint32_t *>(p);
  return (uint64_t)q[0] | ((uint64_t)q[1] << 32);
}

__device__ inline uint32_t rl32(uint32_t v, int k) { return __builtin_amdgcn_readlane(v, k); }
__device__ inline uint64_t rl64(uint64_t v, int k) {
  return (uint64_t)rl32((uint32_t)v, k) | ((uint64_t)rl32((uint32_t)(v >> 32), k) << 32);
}

struct SecView {
  const uint8_t *p;
  uint32_t npts, W, NE, NX, nch, ntile;
  uint64_t A, Poff, Moff, Xoff, sz;
  bool ok;
};

// Locates section (b, l) and checks its structure against the expected
// point count and its table size.
__device__ inline SecView open_section(const DecPlan &D, int64_t b, int l, uint32_t expect_npts) {
  SecView v;
  v.ok = false;
  const int L = D.g.nL - 1;
  const uint64_t ent = kHeaderBytes + 16 * ((uint64_t)b * D.g.nL + (uint64_t)(L - l));
  if (ent + 16 > D.sbytes) return v;
  const uint64_t off = ld64(D.s + ent), sz = ld64(D.s + ent + 8);
  if (off < D.payload_off || (off & 7) || sz < 16 || off + sz > D.sbytes) return v;
  v.p = D.s + off;
  v.npts = ld32(v.p);
  v.W = ld32(v.p + 4);
  v.NE = ld32(v.p + 8);
  v.NX = ld32(v.p + 12);
  if (v.npts != expect_npts) return v;
  if (sec_bytes(v.npts, v.W, v.NE, v.NX) != sz) return v;
  v.nch = (v.npts + 63) / 64;
  v.ntile = (v.nch + 63) / 64;
  v.A = 16 + pad8(12 * (uint64_t)v.ntile);
  v.Poff = v.A + pad8(v.nch);
  v.Moff = v.Poff + 8 * (uint64_t)v.W;
  v.Xoff = v.Moff + 8 * (uint64_t)v.NE;
  v.ok = true;
  return v;
}

// A zero the compiler cannot see through, in a vector register: a uniform
// load at an address offset by it goes through the vector memory path, whose
// wait counter it does not share with the kernel's scalar loads (of its
// arguments, say), so a later scalar load's wait does not wait for it.
__device__ inline uint32_t vzero() {
  uint32_t z = 0u;
  asm volatile("" : "+v"(z));
  return z;
}

// Section (b, l) located from its table entry alone, for a reader that
// issues its tile-table and chunk-header loads before the section's own
// header arrives: the layout up to the payload comes from the expected point
// count (checked to fit in the section), `ok` covers the entry and that fit,
// and the header's fields (loaded here through the vector path, not yet
// used) are checked by sec_fields_ok; Moff and Xoff are left to the caller.
__device__ inline SecView open_section_early(const DecPlan &D, int64_t b, int l, uint32_t expect_npts) {
  SecView v;
  v.ok = false;
  const int L = D.g.nL - 1;
  const uint64_t ent = kHeaderBytes + 16 * ((uint64_t)b * D.g.nL + (uint64_t)(L - l));
  if (ent + 16 > D.sbytes) return v;
  const uint64_t off = ld64(D.s + ent), sz = ld64(D.s + ent + 8);
  if (off < D.payload_off || (off & 7) || sz < 16 || off + sz > D.sbytes) return v;
  v.p = D.s + off;
  v.sz = sz;
  v.nch = (expect_npts + 63) / 64;
  v.ntile = (v.nch + 63) / 64;
  v.A = 16 + pad8(12 * (uint64_t)v.ntile);
  v.Poff = v.A + pad8(v.nch);
  if (v.Poff > sz) return v;
  const uint8_t *hp = v.p + vzero();
  v.npts = ld32(hp);
  v.W = ld32(hp + 4);
  v.NE = ld32(hp + 8);
  v.NX = ld32(hp + 12);
  v.ok = true;
  return v;
}

// The checks open_section makes on a section's header fields.
__device__ inline bool sec_fields_ok(const SecView &v, uint32_t expect_npts) {
  return v.npts == expect_npts && sec_bytes(v.npts, v.W, v.NE, v.NX) == v.sz;
}

// Block activity flags of a differentiated stream: bit 0 of the spare word
// of each block-table record (stride 4 words).
__device__ inline NearSel dec_near(const DecPlan &D, int64_t b, const int64_t o[3], const int64_t hi[3]) {
  const Geo &g = D.g;
  const uint32_t *act =
      reinterpret_cast<const uint32_t *>(D.s + kHeaderBytes + 16 * (uint64_t)g.nblocks * (uint64_t)g.nL + 12);
  return near_sel(g, act, 4u, b, o, hi);
}

__device__ inline void set_status(const DecPlan &D, int32_t code) {
  if (D.status) atomicMin(D.status, code);
}

// Block-table range [min, max] of block b's reconstructed values.
__device__ inline void block_range(const DecPlan &D, int64_t b, float &mn, float &mx) {
  const uint64_t off = kHeaderBytes + 16 * ((uint64_t)D.g.nblocks * D.g.nL + (uint64_t)b);
  mn = __uint_as_float(ld32(D.s + off));
  mx = __uint_as_float(ld32(D.s + off + 4));
}

// Whether block b is reconstructed: always, unless the reconstruction is
// restricted to isovalues k in [kmin, kmax]; then only blocks whose range
// gives min < k <= max for some such k (the others hold no cell whose
// corners lie on both sides of any such k).
__device__ inline bool block_needed(const DecPlan &D, int64_t b) {
  if (!D.prune) return true;
  float mn, mx;
  block_range(D, b, mn, mx);
  return mn < mx && mn < D.kmax && D.kmin <= mx;
}

// Decodes chunks [kbeg, kend) of tile t of a section (every lane of the
// wave takes part in the tile's offset scan); calls emit(z, y, x, value) for
// every point.
template <class Emit>
__device__ void dec_tile(const DecPlan &D, const SecView &v, int l, const int64_t o[3], const NearSel &ns, const Sec &s,
                         uint32_t t, uint32_t kbeg, uint32_t kend, Emit emit) {
  const Geo &g = D.g;
  const int L = g.nL - 1;
  const int lane = lane_id();
  const uint32_t c = t * 64 + (uint32_t)lane;
  const uint8_t *tt = v.p + 16 + 12 * (uint64_t)t;
  const uint32_t tw = ld32(tt), te = ld32(tt + 4), tx = ld32(tt + 8);
  const uint32_t hb = c < v.nch ? v.p[v.A + c] : 0u;
  const uint32_t w = hb & 31u, he = hb >> 7;
  const uint32_t wo = tw + wave_excl_sum_dpp(w), eo = te + wave_excl_sum_dpp(he);
  // structural checks: widths, exact masks and values stay inside the section
  const uint32_t bad_l = (w > (uint32_t)kMaxW) || (hb & 0x60u) || (wo + w > v.W) || (he && eo >= v.NE);
  if (__ballot(bad_l)) {
    set_status(D, -4);
    return;
  }
  const uint64_t em = he ? ld64(v.p + v.Moff + 8 * (uint64_t)eo) : 0ull;
  const uint32_t pc = (uint32_t)__popcll(em);
  const uint32_t xo = tx + wave_excl_sum_dpp(pc);
  if (__ballot(xo + pc > v.NX)) {
    set_status(D, -4);
    return;
  }
  const uint32_t nc = min(min(64u, v.nch - t * 64), kend);
  const float *Gp = (l < L) ? D.gp[l + 1] : nullptr;
  const uint32_t g0 = (uint32_t)D.gd[l + 1][0], g1 = (uint32_t)D.gd[l + 1][1], g2 = (uint32_t)D.gd[l + 1][2];
  for (uint32_t k = kbeg; k < nc; k++) {
    const uint32_t wk = rl32(w, (int)k), wok = rl32(wo, (int)k), xok = rl32(xo, (int)k);
    const uint64_t emk = rl64(em, (int)k);
    const uint32_t j = (t * 64 + k) * 64 + (uint32_t)lane;
    if (j >= s.npts) continue;
    uint32_t zc = 0;
    if (wk) {
      const uint32_t bit = (uint32_t)lane * wk, off = bit & 31u;
      const uint8_t *wp = v.p + v.Poff + 8 * (uint64_t)wok + 4 * (uint64_t)(bit >> 5);
      uint32_t lo = ld32(wp);
      zc = lo >> off;
      if (off + wk > 32u) zc |= ld32(wp + 4) << (32u - off);
      zc &= (wk == 32u) ? 0xffffffffu : ((1u << wk) - 1u);
    }
    uint32_t ww, vv, uu;
    sec_point(s, j, ww, vv, uu);
    const uint32_t z = (uint32_t)o[0] + (ww << l), y = (uint32_t)o[1] + (vv << l), x = (uint32_t)o[2] + (uu << l);
    float r;
    if ((emk >> lane) & 1ull) {
      r = __uint_as_float(ld32(v.p + v.Xoff + 4 * ((uint64_t)xok + lanes_below(emk))));
    } else {
      const float p = (l == L) ? 0.0f : predict(Gp, g0, g1, g2, l, z, y, x);
      const int32_t q = (int32_t)(zc >> 1) ^ -(int32_t)(zc & 1u);
      const QuantP qp = quant_pick(g, g.diff && !near_at(ns, z, y, x));
      r = qp.lossless ? p : __fadd_rn(p, __fmul_rn((float)q, qp.step));
    }
    emit(z, y, x, r);
  }
}

// Coarse levels of one block per workgroup.
__global__ __launch_bounds__(kBS) void k_decode_coarse(DecPlan D) {
  const Geo &g = D.g;
  const int L = g.nL - 1;
  const int64_t b = blockIdx.x;
  if (!block_needed(D, b)) return;
  const int wave = threadIdx.x / kWave;
  const int lmin = D.lo > 3 ? D.lo : 3;  // levels 2 and 1 have wide kernels of their own
  int64_t o[3], hi[3];
  unit_ext(g, b, o, hi);
  const NearSel ns = g.diff ? dec_near(D, b, o, hi) : NearSel{};
  for (int l = L; l >= lmin; l--) {
    float *dst = D.gp[l];
    const int64_t *gd = D.gd[l];
    if (l < L) {
      const int sh = l + 1;
      const uint32_t c0 = (uint32_t)((hi[0] - o[0]) >> sh) + 1, c1 = (uint32_t)((hi[1] - o[1]) >> sh) + 1;
      const uint32_t c2 = (uint32_t)((hi[2] - o[2]) >> sh) + 1;
      const float *src = D.gp[l + 1];
      const uint32_t zo = (uint32_t)(o[0] >> sh), yo = (uint32_t)(o[1] >> sh), xo = (uint32_t)(o[2] >> sh);
      const uint32_t s1 = (uint32_t)D.gd[l + 1][1], s2 = (uint32_t)D.gd[l + 1][2];
      const uint32_t d1 = (uint32_t)gd[1], d2 = (uint32_t)gd[2];
      for (uint32_t r = wave; r < c0 * c1; r += kWaves) {
        const uint32_t w = r / c1, v = r - (r / c1) * c1;
        const size_t srow = ((size_t)(zo + w) * s1 + (yo + v)) * s2 + xo;
        const size_t drow = ((size_t)(2 * (zo + w)) * d1 + 2 * (yo + v)) * d2 + 2 * xo;
        for (uint32_t u = lane_id(); u < c2; u += kWave) dst[drow + 2 * u] = src[srow + u];
      }
    }
    const Sec s = sec_geom(o, hi, l, L);
    const SecView v = open_section(D, b, l, s.npts);
    if (!v.ok) {
      if (threadIdx.x == 0) set_status(D, -4);
    } else {
      for (uint32_t t = wave; t < v.ntile; t += kWaves)
        dec_tile(D, v, l, o, ns, s, t, 0u, 64u, [&](uint32_t z, uint32_t y, uint32_t x, float r) {
          dst[((size_t)(z >> l) * (uint32_t)gd[1] + (y >> l)) * (uint32_t)gd[2] + (x >> l)] = r;
        });
    }
    __syncthreads();
  }
}

// Level 0 over (tile groups, blocks): each wave decodes one tile and writes
// the points the block owns, plus the coarse (even) points of even rows.
__global__ __launch_bounds__(kBS) void k_decode_fine(DecPlan D) {
  const Geo &g = D.g;
  const int L = g.nL - 1;
  const int64_t b = blockIdx.y;
  if (!block_needed(D, b)) return;
  const uint32_t t = blockIdx.x * kWaves + threadIdx.x / kWave;
  int64_t o[3], hi[3];
  unit_ext(g, b, o, hi);
  const Sec s = sec_geom(o, hi, 0, L);
  const uint32_t nch = (s.npts + 63) / 64;
  if (t >= (nch + 63) / 64) return;
  const SecView v = open_section(D, b, 0, s.npts);
  if (!v.ok) {
    if (lane_id() == 0) set_status(D, -4);
    return;
  }
  const int64_t n1 = g.n[1], n2 = g.n[2];
  const int64_t ez = (hi[0] < g.n[0] - 1) ? hi[0] : g.n[0];  // first z not owned
  const int64_t ey = (hi[1] < g.n[1] - 1) ? hi[1] : g.n[1];
  const int64_t ex = (hi[2] < g.n[2] - 1) ? hi[2] : g.n[2];
  const float *G1 = (L >= 1) ? D.gp[1] : nullptr;
  const int64_t *gd1 = D.gd[1];
  float *out = D.out;
  // each block writes the points it owns -- or, in a restricted
  // reconstruction, its whole closed extent (a neighbour owning the shared
  // faces may be left out; both write identical values where both run)
  const bool all = D.prune != 0;
  const NearSel ns = g.diff ? dec_near(D, b, o, hi) : NearSel{};
  dec_tile(D, v, 0, o, ns, s, t, 0u, 64u, [&](uint32_t z, uint32_t y, uint32_t x, float r) {
    if (!all && (z >= ez || y >= ey)) return;
    float *row = out + ((size_t)z * (uint32_t)n1 + y) * (uint32_t)n2;
    if (all || x < ex) row[x] = r;
    if (L >= 1 && !((z | y) & 1u) && (x & 1u)) {
      // even row of an even plane: the neighbouring even points come from level 1
      const float *g1 = G1 + ((size_t)(z >> 1) * (uint32_t)gd1[1] + (y >> 1)) * (uint32_t)gd1[2];
      row[x - 1] = g1[(x - 1) >> 1];
      if (x + 1 == hi[2] && (all || hi[2] == g.n[2] - 1)) row[x + 1] = g1[(x + 1) >> 1];
    }
  });
}

// Level 1 (nL >= 2) over (tiles, blocks): one workgroup per tile, each wave
// 16 of its chunks; the block's level-2 points are copied into the level-1
// grid (the output when level 1 is requested) by the same workgroups.
// One level l in {1, 2} of every block: workgroup (t, b) decodes tile t of
// block b's level-l section (16 chunks per wave) after carrying the block's
// level-(l+1) points over into the level-l compact grid.
__global__ __launch_bounds__(kBS) void k_decode_level(DecPlan D, int l) {
  const Geo &g = D.g;
  const int L = g.nL - 1;
  uint32_t t, b;
  xcd_remap(t, b);
  if (!block_needed(D, b)) return;
  const int wave = threadIdx.x / kWave;
  int64_t o[3], hi[3];
  int cls = 0;
  if (g.units) {
    unit_ext(g, b, o, hi);
  } else {
    const BlockPos bp = block_pos(g, D.l0, b);
    for (int a = 0; a < 3; a++) { o[a] = bp.o[a]; hi[a] = bp.hi[a]; }
    cls = bp.cls;
  }
  float *dst = D.gp[l];
  const int64_t *gd = D.gd[l];
  if (l < L) {
    const int sh = l + 1;
    const uint32_t c0 = (uint32_t)((hi[0] - o[0]) >> sh) + 1, c1 = (uint32_t)((hi[1] - o[1]) >> sh) + 1;
    const uint32_t c2 = (uint32_t)((hi[2] - o[2]) >> sh) + 1;
    const float *src = D.gp[l + 1];
    const uint32_t zo = (uint32_t)(o[0] >> sh), yo = (uint32_t)(o[1] >> sh), xo = (uint32_t)(o[2] >> sh);
    const uint32_t s1 = (uint32_t)D.gd[l + 1][1], s2 = (uint32_t)D.gd[l + 1][2];
    const uint32_t d1 = (uint32_t)gd[1], d2 = (uint32_t)gd[2];
    // one row of the coarser block grid per wave step
    for (uint32_t r = t * kWaves + wave; r < c0 * c1; r += gridDim.x * kWaves) {
      const uint32_t w = r / c1, v = r - (r / c1) * c1;
      const size_t srow = ((size_t)(zo + w) * s1 + (yo + v)) * s2 + xo;
      const size_t drow = ((size_t)(2 * (zo + w)) * d1 + 2 * (yo + v)) * d2 + 2 * xo;
      for (uint32_t u = lane_id(); u < c2; u += kWave) dst[drow + 2 * u] = src[srow + u];
    }
  }
  const Sec s = (l == 1 && !g.units) ? D.l0.sec1[cls] : sec_geom(o, hi, l, L);
  const uint32_t nch = (s.npts + 63) / 64;
  if (t >= (nch + 63) / 64) return;
  const SecView v = open_section(D, b, l, s.npts);
  if (!v.ok) {
    if (threadIdx.x == 0) set_status(D, -4);
    return;
  }
  const int lv = l;
  const NearSel ns = g.diff ? dec_near(D, b, o, hi) : NearSel{};
  dec_tile(D, v, l, o, ns, s, t, wave * 16u, wave * 16u + 16u, [&](uint32_t z, uint32_t y, uint32_t x, float r) {
    dst[((size_t)(z >> lv) * (uint32_t)gd[1] + (y >> lv)) * (uint32_t)gd[2] + (x >> lv)] = r;
  });
}

// Levels 0, 1 and 2 below a coarser level (level LV + 1 exists) over (tile
// groups, blocks), for block shapes whose index products fit 24 bits: each
// wave decodes CPW consecutive chunks of one tile (P.cpw0 at level 0, 16
// above), with block geometry and reciprocals from the host-filled shape
// table and block-relative 32-bit offsets from uniform base pointers (the
// block's first plane of the output and of the parent grid).  Level 0 writes
// the points the block owns plus the even points of even rows taken from
// level 1; levels 1 and 2 write every point of their section into grid LV,
// after carrying the block's points of grid LV + 1 over into it.
template <int LV, bool DIFF>
__device__ __forceinline__ void decode_fast(const DecPlan &D) {
  const Geo &g = D.g;
  uint32_t gxi, b;
  xcd_remap(gxi, b);
  if (!block_needed(D, b)) return;
  const uint32_t wave = wave_index();
  const int lane = lane_id();
  const BlockPos bp = block_pos(g, D.l0, b);
  if (LV >= 1) {
    // one row of the block's grid LV + 1 per wave step
    constexpr int sh = LV + 1;
    const uint32_t c0 = ((bp.hi[0] - bp.o[0]) >> sh) + 1, c1 = ((bp.hi[1] - bp.o[1]) >> sh) + 1;
    const uint32_t c2 = ((bp.hi[2] - bp.o[2]) >> sh) + 1;
    const float *src = D.gp[LV + 1];
    float *dst = D.gp[LV];
    const uint32_t zo = bp.o[0] >> sh, yo = bp.o[1] >> sh, xo = bp.o[2] >> sh;
    const uint32_t s1 = (uint32_t)D.gd[LV + 1][1], s2 = (uint32_t)D.gd[LV + 1][2];
    const uint32_t d1 = (uint32_t)D.gd[LV][1], d2 = (uint32_t)D.gd[LV][2];
    for (uint32_t r = gxi * kWaves + wave; r < c0 * c1; r += gridDim.x * kWaves) {
      const uint32_t w = r / c1, v = r - w * c1;
      const size_t srow = ((size_t)(zo + w) * s1 + (yo + v)) * s2 + xo;
      const size_t drow = ((size_t)(2 * (zo + w)) * d1 + 2 * (yo + v)) * d2 + 2 * xo;
      for (uint32_t u = (uint32_t)lane; u < c2; u += kWave) dst[drow + 2 * u] = src[srow + u];
    }
  }
  const uint32_t cpw = LV == 0 ? (uint32_t)D.cpw0 : 16u;
  const uint32_t cbeg = (gxi * kWaves + wave) * cpw;  // first chunk of this wave
  const uint32_t t = cbeg >> 6, kbeg = cbeg & 63u;
  const Sec s = LV == 0 ? D.l0.sec[bp.cls] : LV == 1 ? D.l0.sec1[bp.cls] : D.l0.sec2[bp.cls];  // scalar registers
  const uint32_t nch = (s.npts + 63) / 64;
  if (t >= (nch + 63) / 64) return;
  const SecView v = open_section(D, b, LV, s.npts);
  if (!v.ok) {
    if (lane == 0) set_status(D, -4);
    return;
  }
  const uint32_t n1 = (uint32_t)g.n[1], n2 = (uint32_t)g.n[2];
  const uint32_t oyl = bp.o[1] >> LV, oxl = bp.o[2] >> LV;
  const uint32_t ownz = bp.own[0] - bp.o[0], owny = bp.own[1], ownx = bp.own[2];
  const bool lastx = (bp.hi[2] == (uint32_t)g.n[2] - 1);
  const bool all = D.prune != 0;
  // output: the field (level 0) or grid LV, from the block's first plane
  const uint32_t f1 = (uint32_t)D.gd[LV][1], f2 = (uint32_t)D.gd[LV][2];
  char *__restrict__ obase = LV == 0 ? reinterpret_cast<char *>(D.out + (size_t)bp.o[0] * n1 * n2)
                                     : reinterpret_cast<char *>(D.gp[LV] + (size_t)(bp.o[0] >> LV) * f1 * f2);
  const uint32_t h0 = (uint32_t)D.gd[LV + 1][0], h1 = (uint32_t)D.gd[LV + 1][1], h2 = (uint32_t)D.gd[LV + 1][2];
  const uint32_t zp = bp.o[0] >> (LV + 1);
  // uniform bases; the launcher guarantees the block's slab spans < 4 GiB
  const char *__restrict__ Pb = reinterpret_cast<const char *>(D.gp[LV + 1] + (size_t)zp * h1 * h2);
  const uint32_t h2x4 = h2 * 4u, h12x4 = h1 * h2 * 4u;
  const float step = g.step;
  const int lossless = g.lossless;
  NearSel ns{};
  bool mixed = false, allfar = false;
  if (DIFF) {
    const int64_t o3[3] = {bp.o[0], bp.o[1], bp.o[2]}, hi3[3] = {bp.hi[0], bp.hi[1], bp.hi[2]};
    ns = dec_near(D, b, o3, hi3);
    mixed = ns.lut != 0u && ns.lut != kNearAll;   // else one quantizer for the whole block
    allfar = ns.lut == 0u;
  }
  // scalar constants of an unmixed block
  const float stepb = DIFF && allfar ? g.step2 : step;
  const int llb = DIFF && allfar ? g.lossless2 : lossless;

  const uint32_t c = t * 64 + (uint32_t)lane;
  const uint8_t *tt = v.p + 16 + 12 * (uint64_t)t;
  const uint32_t tw = ld32(tt), te = ld32(tt + 4), tx = ld32(tt + 8);
  const uint32_t hb = c < v.nch ? v.p[v.A + c] : 0u;
  const uint32_t w = hb & 31u, he = hb >> 7;
  const uint32_t wo = tw + wave_excl_sum_dpp(w), eo = te + wave_excl_sum_dpp(he);
  const uint32_t bad_l = (w > (uint32_t)kMaxW) || (hb & 0x60u) || (wo + w > v.W) || (he && eo >= v.NE);
  if (__ballot(bad_l)) {
    set_status(D, -4);
    return;
  }
  const uint64_t em = he ? ld64(v.p + v.Moff + 8 * (uint64_t)eo) : 0ull;
  const uint32_t pc = (uint32_t)__popcll(em);
  const uint32_t xo = tx + wave_excl_sum_dpp(pc);
  if (__ballot(xo + pc > v.NX)) {
    set_status(D, -4);
    return;
  }
  const uint32_t nc = min(min(64u, v.nch - t * 64), kbeg + cpw);
  const char *__restrict__ payb = reinterpret_cast<const char *>(v.p + v.Poff);
  const char *__restrict__ exvb = reinterpret_cast<const char *>(v.p + v.Xoff);
  const SecR rc = LV == 0 ? D.l0.rc[bp.cls] : LV == 1 ? D.l0.rc1[bp.cls] : D.l0.rc2[bp.cls];
  const uint32_t jmax = s.npts - 1;  // npts > 0: this wave's tile holds a chunk
  const uint32_t hi2 = bp.hi[2];
  // kDecGroup chunks at a time: coordinates and addresses of all of them,
  // then every load (the eight parents of each point, payload words, exact
  // values), then every value is computed before any store, so no load is
  // left pending on a path and no store sits between a load and its use.  A
  // chunk past the wave's range repeats the last one and lanes past the
  // section read a clamped point; neither is written.
#pragma unroll 1
  for (uint32_t k0 = kbeg; k0 < nc; k0 += kDecGroup) {
    float pa[kDecGroup][8], r[kDecGroup];
    uint32_t pw0[kDecGroup], pw1[kDecGroup], xv[kDecGroup], orow[kDecGroup], off[kDecGroup];
    bool zu[kDecGroup], yu[kDecGroup], xu[kDecGroup], ex[kDecGroup], wr[kDecGroup], wx[kDecGroup], ev[kDecGroup],
        e1[kDecGroup], far[kDecGroup];
#pragma unroll
    for (int u = 0; u < kDecGroup; u++) {
      const uint32_t k = min(k0 + (uint32_t)u, nc - 1);
      const uint32_t wk = rl32(w, (int)k), wok = rl32(wo, (int)k), xok = rl32(xo, (int)k);
      const uint64_t emk = rl64(em, (int)k);
      const uint32_t jr = (t * 64 + k) * 64 + (uint32_t)lane;
      uint32_t zz_, vv, uu;
      sec_point24(s, rc, min(jr, jmax), zz_, vv, uu);
      // (zz_, V, U): the point on the level-LV grid (zz_ relative to the block)
      const uint32_t V = oyl + vv, U = oxl + uu;
      far[u] = DIFF && mixed && !near_at(ns, bp.o[0] + (zz_ << LV), V << LV, U << LV);
      const uint32_t zl = zz_ >> 1, yl = V >> 1, xl = U >> 1;
      zu[u] = (zz_ & 1u) && (zp + zl + 1 < h0);
      yu[u] = (V & 1u) && (yl + 1 < h1);
      xu[u] = (U & 1u) && (xl + 1 < h2);
      const uint32_t o00 = mad24s(mad24s(zl, h1, yl), h2, xl) * 4u;
      const uint32_t dxo = xu[u] ? 4u : 0u, dyo = yu[u] ? h2x4 : 0u, dzo = zu[u] ? h12x4 : 0u;
      const uint32_t o01 = o00 + dyo, o10 = o00 + dzo, o11 = o10 + dyo;
      pa[u][0] = ldf(Pb, o00); pa[u][1] = ldf(Pb, o00 + dxo);
      pa[u][2] = ldf(Pb, o01); pa[u][3] = ldf(Pb, o01 + dxo);
      pa[u][4] = ldf(Pb, o10); pa[u][5] = ldf(Pb, o10 + dxo);
      pa[u][6] = ldf(Pb, o11); pa[u][7] = ldf(Pb, o11 + dxo);
      const uint32_t bit = mul24s((uint32_t)lane, wk);
      off[u] = bit & 31u;
      pw0[u] = 0u;
      pw1[u] = 0u;
      if (wk) {
        const uint32_t wb = 8u * wok + 4u * (bit >> 5);
        pw0[u] = ldu(payb, wb);
        pw1[u] = ldu(payb, wb + ((off[u] + wk > 32u) ? 4u : 0u));
      }
      ex[u] = (emk >> lane) & 1ull;
      xv[u] = 0u;
      if (ex[u]) xv[u] = ldu(exvb, 4u * (xok + lanes_below(emk)));
      const bool valid = (k0 + (uint32_t)u < nc) && (jr < s.npts);
      if (LV == 0) {
        // the points the block owns -- or, in a restricted reconstruction,
        // its whole closed extent (a neighbour owning the shared faces may
        // be left out; both write identical values where both run)
        wr[u] = valid && (all || (zz_ < ownz && V < owny));
        wx[u] = all || U < ownx;
        // even row of an even plane: the neighbouring even points come from
        // level 1 (they are this point's two x parents)
        ev[u] = !((zz_ | V) & 1u) && (U & 1u);
        e1[u] = U + 1 == hi2 && (lastx || all);
        orow[u] = (mul24s(mad24s(zz_, n1, V), n2) + U) * 4u;
      } else {
        wr[u] = valid;
        wx[u] = true;
        ev[u] = false;
        e1[u] = false;
        orow[u] = mad24s(mad24s(zz_, f1, V), f2, U) * 4u;
      }
    }
#pragma unroll
    for (int u = 0; u < kDecGroup; u++) {
      const uint32_t wk = rl32(w, (int)min(k0 + (uint32_t)u, nc - 1));
      const float p = midpoint8(pa[u][0], pa[u][1], pa[u][2], pa[u][3], pa[u][4], pa[u][5], pa[u][6], pa[u][7],
                                zu[u], yu[u], xu[u]);
      const uint32_t o = off[u];
      uint32_t zc = (o + wk > 32u) ? ((pw0[u] >> o) | (pw1[u] << (32u - o))) : (pw0[u] >> o);
      zc = wk ? (zc & ((1u << wk) - 1u)) : 0u;
      const int32_t q = (int32_t)(zc >> 1) ^ -(int32_t)(zc & 1u);
      const float st = DIFF && far[u] ? g.step2 : stepb;
      const int ll = DIFF && far[u] ? g.lossless2 : llb;
      const float rq = ll ? p : __fadd_rn(p, __fmul_rn((float)q, st));
      r[u] = ex[u] ? __uint_as_float(xv[u]) : rq;
      hold(r[u]);
      hold(pa[u][0]);
      hold(pa[u][1]);
    }
#pragma unroll
    for (int u = 0; u < kDecGroup; u++) {
      if (!wr[u]) continue;
      const uint32_t ro = orow[u];
      if (wx[u]) stf(obase, ro, r[u]);
      if (LV == 0 && ev[u]) {
        stf(obase, ro - 4u, pa[u][0]);
        if (e1[u]) stf(obase, ro + 4u, pa[u][1]);
      }
    }
  }
}

// ------------------------------------------------------- level 0 by plane pairs
//
// Reconstruction of level 0 of 64-cell blocks (at most 65 points per axis)
// below a coarser level, one workgroup per (pair of z-planes, block) -- the
// compression kernel's tiling.  The workgroup stages the two level-1 planes
// that hold the pair's parents in LDS, reads the headers, exact masks and
// exact-value offsets of the chunks that overlap the pair's part of the
// section, unpacks their codes into LDS at their section positions (payload
// words, masks and exact values are all loaded before any store), and then
// writes the pair's field rows along x (lane = point): level-0 points from
// their prediction and code, the even points of even rows of the even plane
// from level 1.  Rows and points the block does not own are not written
// (in a restricted reconstruction the whole closed extent is).

constexpr int kD0Side = 33;                  // level-1 points per axis of a 64-cell block
constexpr int kD0Plane = 1152;               // staged plane stride (floats; fits an LDS immediate offset)
constexpr int kD0Codes = 7361;               // most section points of a pair
constexpr int kD0Chunks = 118;               // chunks that overlap a pair's part of the section
constexpr int kD0Xcap = 128;                 // exact values of a pair staged in LDS (more are read from the stream)
constexpr int kD0Group = 8;                  // pairs of chunks (unpack) whose loads a wave issues together
constexpr int kD0Rows = 8;                   // rows a wave reconstructs before storing any
constexpr int32_t kD0ExactQ = -32768;        // LDS code of a point stored exactly (codes are within +-32767)

struct D0Ctx {
  const int16_t *sc;
  const uint32_t *cxo;
  const unsigned long long *cem;
  const float *xl;
  const uint8_t *xs;       // exact values of the section in the stream
  uint32_t J0, c0, xo0;
  float step;
};

// Value of a level-0 point predicted as p whose (signed) LDS code is q (not
// an exact point).
__device__ __forceinline__ float d0_quant(const D0Ctx &t, int32_t q, float p) {
  return __fadd_rn(p, __fmul_rn((float)q, t.step));
}

// The exact value of the level-0 point at section index j: the (rank within
// its chunk)-th exact value of the chunk.
__device__ __forceinline__ float d0_exact(const D0Ctx &t, uint32_t j) {
  const uint32_t k = (j >> 6) - t.c0;
  const unsigned long long em = t.cem[k];
  const uint32_t ix = t.cxo[k] + (uint32_t)__popcll(em & ((1ull << (j & 63u)) - 1ull));
  if (ix - t.xo0 < (uint32_t)kD0Xcap) return t.xl[ix - t.xo0];
  return __uint_as_float(ld32(t.xs + 4 * (uint64_t)ix));
}

__device__ __forceinline__ float d0_xavg(float a0, float a1, bool xav) {
  float m = avg2(a0, a1);
  hold(m);
  return xav ? m : a0;
}

__device__ __forceinline__ float d0_lds(const char *base, uint32_t off) {
  return *reinterpret_cast<const float *>(base + off);
}

// Marching cubes' below-isovalue words of a group of kD0Rows decoded rows
// along x: the word of row k for isovalue j is computed by the whole wave
// (a ballot) and parked in lane 8 (j mod 8) + k of word set j / 8; then each
// lane stores its word (at most two stores per group, for 16 isovalues).
struct D0Bits {
  uint32_t lo[2], hi[2];
};

// Words of the group's rows for isovalues j in [j0, j1) (j1 - j0 <= 8) into
// one word set: isovalue j, row k at lane 8 (j - j0) + k.
__device__ __forceinline__ void d0_bits_set(const DecPlan &D, uint32_t &lo, uint32_t &hi, const float (&rv)[kD0Rows],
                                            int j0, int j1, unsigned long long vmask) {
  for (int j = j0; j < j1; j++) {
    const float kj = D.kb[j];
    const uint32_t L0 = 8u * (uint32_t)(j - j0);
#pragma unroll
    for (int k = 0; k < kD0Rows; k++) {
      const unsigned long long m = __ballot(rv[k] < kj) & vmask;
      writelane(lo, (uint32_t)m, L0 + (uint32_t)k);
      writelane(hi, (uint32_t)(m >> 32), L0 + (uint32_t)k);
    }
  }
}

__device__ __forceinline__ void d0_bits_rows(const DecPlan &D, D0Bits &q, const float (&rv)[kD0Rows], int nk,
                                             unsigned long long vmask) {
  d0_bits_set(D, q.lo[0], q.hi[0], rv, 0, min(nk, 8), vmask);
  if (nk > 8) d0_bits_set(D, q.lo[1], q.hi[1], rv, 8, nk, vmask);
}

// Level LV (0 or 1) of 64-cell blocks by pairs of planes of the level's
// grid: at level 1 the rows have at most 33 points (lanes past 33 idle), the
// parents come from the level-2 grid and the rows go to the level-1 grid (the
// even points of the even plane's even rows from level 2); no bit planes.
template <int LV>
struct DTileDims {
  static constexpr int Side = (64 >> (LV + 1)) + 1;       // parent points per axis of a block
  static constexpr int Plane = LV == 0 ? kD0Plane : 320;  // staged parent plane stride (floats)
  static constexpr int Codes = LV == 0 ? kD0Codes : 1889; // most section points of a pair
  static constexpr int Chunks = LV == 0 ? kD0Chunks : 32; // chunks that overlap a pair's part of the section
};

template <int LV>
__device__ __forceinline__ void decode_tile(const DecPlan &D) {
  using TD = DTileDims<LV>;
  constexpr uint32_t S = 1u << LV;             // field points per level step
  __shared__ float sg[2 * TD::Plane];
  // signed codes by section index - 64 c0 (c0 the pair's first chunk): the
  // pair's first and last chunks unpack whole (at most 63 points before J0
  // and 63 after J1), and a last pair of chunks may end one chunk past them
  __shared__ __align__(4) int16_t scs[TD::Codes + 192];
  // chunk headers: width | payload byte offset << 5 (zero-width entries for
  // the 64 chunks past the range, which the unpacking's last pairs read),
  // exact-value offsets and exact masks (a zero entry past the range)
  __shared__ uint32_t cwh[TD::Chunks + 64], cxo[TD::Chunks + 1];
  __shared__ unsigned long long cem[TD::Chunks + 1];
  __shared__ float xl[kD0Xcap];
  __shared__ uint32_t sbad[kWaves];
  uint32_t w2, b;
  xcd_remap(w2, b);
  if (!block_needed(D, b)) return;
  const Geo &g = D.g;
  const BlockPos bp = block_pos(g, D.l0, b);
  const Sec s = LV == 0 ? D.l0.sec[bp.cls] : D.l0.sec1[bp.cls];
  const uint32_t PP = s.Pe + s.Po, J0 = w2 * PP;
  if (J0 >= s.npts) return;
  const uint32_t we = 2 * w2;
  const bool all = D.prune != 0;
  const uint32_t ownz = bp.own[0] - bp.o[0], owny = bp.own[1] - bp.o[1], ownx = bp.own[2] - bp.o[2];
  if (!all && we * S >= ownz) return;          // neither plane of the pair is the block's
  const bool has_odd = we + 1 < s.mz;
  const uint32_t J1 = has_odd ? J0 + PP : J0 + s.Pe;
  const uint32_t c0 = J0 >> 6, c1 = (J1 + 63) >> 6, ncw = c1 - c0;
  const uint32_t wave = wave_index();
  const int lane = lane_id();
  const uint32_t n1 = (uint32_t)g.n[1], n2 = (uint32_t)g.n[2];
  const uint32_t mx = s.mx, my = s.my, rowE = s.rowE, RP = rowE + mx;
  const uint32_t h0 = (uint32_t)D.gd[LV + 1][0], h1 = (uint32_t)D.gd[LV + 1][1], h2 = (uint32_t)D.gd[LV + 1][2];
  const uint32_t zl0 = (bp.o[0] >> (LV + 1)) + w2, oy1 = bp.o[1] >> (LV + 1), ox1 = bp.o[2] >> (LV + 1);
  const uint32_t gy = (bp.hi[1] >> (LV + 1)) - oy1 + 1, gx = (bp.hi[2] >> (LV + 1)) - ox1 + 1;
  const uint32_t np = zl0 + 1 < h0 ? 2u : 1u;
  // The loads overlap: the parent planes first (rows past the block and
  // lanes past a row load, and later store, a copy of the last one; without
  // an upper plane the second staged plane is a copy of the first and is
  // never read), then the section's table entry, then together the section's
  // header, its tile table and the chunk headers of the range (offsets from
  // the block's geometry), then the exact masks; the parents reach LDS last.
  const uint32_t xl1 = min((uint32_t)lane, gx - 1);
  constexpr int kRP = (TD::Side + kWaves - 1) / kWaves;
  float tv[2][kRP];
  {
    const char *__restrict__ g1b =
        reinterpret_cast<const char *>(D.gp[LV + 1] + ((size_t)zl0 * h1 + oy1) * h2 + ox1);
    const uint32_t planeB = (np - 1) * h1 * h2 * 4u, rowB1 = h2 * 4u;
#pragma unroll
    for (int pz = 0; pz < 2; pz++)
#pragma unroll
      for (int u = 0; u < kRP; u++) {
        const uint32_t yy = min(wave + (uint32_t)u * kWaves, gy - 1);
        tv[pz][u] = ldf(g1b, (uint32_t)pz * planeB + yy * rowB1 + xl1 * 4u);
      }
  }
  const SecView v = open_section_early(D, b, LV, s.npts);
  if (!v.ok) {
    if (threadIdx.x == 0) set_status(D, -4);
    return;
  }
  {
    // chunk headers of the (at most three) 64-chunk tiles of the range:
    // widths, payload offsets, exact masks and exact-value offsets, with the
    // structural checks of every reader of a section
    const uint32_t t = (c0 >> 6) + wave;
    uint32_t bad = 0u;
    if (t <= ((c1 - 1) >> 6)) {
      const uint32_t c = t * 64 + (uint32_t)lane;
      const uint8_t *tt = v.p + 16 + 12 * (uint64_t)t + vzero();
      const uint32_t tw = ld32(tt), te = ld32(tt + 4), tx = ld32(tt + 8);
      const uint32_t hb = c < v.nch ? v.p[v.A + c] : 0u;
      const bool fok = sec_fields_ok(v, s.npts);
      const uint64_t Moff = v.Poff + 8 * (uint64_t)v.W;
      const uint32_t w = hb & 31u, he = hb >> 7;
      const uint32_t wo = tw + wave_excl_sum_dpp(w), eo = te + wave_excl_sum_dpp(he);
      const bool badl = !fok || (w > (uint32_t)kMaxW) || (hb & 0x60u) || (wo + w > v.W) || (he && eo >= v.NE);
      const unsigned long long em = (he && !badl) ? ld64(v.p + Moff + 8 * (uint64_t)eo) : 0ull;
      const uint32_t pc = (uint32_t)__popcll(em);
      const uint32_t xo = tx + wave_excl_sum_dpp(pc);
      bad = __ballot(badl || xo + pc > v.NX) != 0ull ? 1u : 0u;
      const bool in = c >= c0 && c < c1;
      bad |= __ballot(in && em != 0ull) != 0ull ? 2u : 0u;
      if (in) {
        cwh[c - c0] = w | (8u * wo) << 5;
        cxo[c - c0] = xo;
        cem[c - c0] = em;
      }
    }
    if (lane == 0) sbad[wave] = bad;
    if (threadIdx.x < 64) cwh[ncw + threadIdx.x] = 0u;
    if (threadIdx.x == 0) cem[ncw] = 0ull;
  }
#pragma unroll
  for (int pz = 0; pz < 2; pz++)
#pragma unroll
    for (int u = 0; u < kRP; u++) {
      const uint32_t yy = min(wave + (uint32_t)u * kWaves, gy - 1);
      sg[pz * TD::Plane + yy * TD::Side + xl1] = tv[pz][u];
    }
  __syncthreads();
  const uint32_t hflags = sbad[0] | sbad[1] | sbad[2] | sbad[3];
  if (hflags & 1u) {
    if (threadIdx.x == 0) set_status(D, -4);
    return;
  }
  const bool tileE = (hflags & 2u) != 0;       // some chunk of the range has exact points
  const uint32_t xo0 = cxo[0];
  const char *__restrict__ payb = reinterpret_cast<const char *>(v.p + v.Poff);
  // the header's fields as uniform values (they arrived before the barrier)
  const uint32_t Wu = (uint32_t)__builtin_amdgcn_readfirstlane((int)v.W);
  const uint32_t NEu = (uint32_t)__builtin_amdgcn_readfirstlane((int)v.NE);
  const uint64_t Xoff = v.Poff + 8 * ((uint64_t)Wu + NEu);
  const char *__restrict__ exb = reinterpret_cast<const char *>(v.p + Xoff);
  // ---- stage the range's exact values (one coalesced pass) and unpack the
  // codes of the pair's points two chunks at a time: for the pair of chunks
  // k = 2i, 2i + 1 of the range, lane l < 32 takes codes 2l, 2l + 1 of chunk
  // k and lane 32 + l those of chunk k + 1 (2 w bits from bit 2 l w of the
  // chunk's payload), decodes both from zigzag form in one word and stores
  // them as one word; each wave issues the payload loads of kD0Group pairs
  // before using any
  {
    const uint32_t nx = min(cxo[ncw - 1] + (uint32_t)__popcll(cem[ncw - 1]) - xo0, (uint32_t)kD0Xcap);
    for (uint32_t i = threadIdx.x; i < nx; i += kBS) xl[i] = __uint_as_float(ldu(exb, 4u * (xo0 + i)));
  }
  {
    const uint32_t lh = (uint32_t)lane & 31u, hf = (uint32_t)lane >> 5;
    const uint32_t npair = (ncw + 1) / 2;
    // the payload and the byte offset of its last word (a section without
    // payload: its own first word, read and not used)
    const char *__restrict__ pldb = Wu ? payb : reinterpret_cast<const char *>(v.p);
    const uint32_t plast = Wu ? 8u * Wu - 4u : 0u;
    for (uint32_t i0 = wave; i0 < npair; i0 += kD0Group * kWaves) {
      uint32_t wu[kD0Group], bu[kD0Group], lo[kD0Group], hi[kD0Group];
#pragma unroll
      for (int u = 0; u < kD0Group; u++) {
        // the lane's chunk (past the range a zero-width entry), and the two
        // payload words its codes can span, loaded without a branch: at
        // offsets clamped to the payload's last word, which changes no word
        // a code uses (a zero-width chunk, or a second word its codes do not
        // reach, reads a word of the payload that is then not used)
        const uint32_t hw = cwh[2 * (i0 + (uint32_t)u * kWaves) + hf];
        const uint32_t w = hw & 31u;
        const uint32_t bit = mul24v(2 * lh, w);
        const uint32_t o0 = min((hw >> 5) + ((bit >> 3) & ~3u), plast);
        wu[u] = w;
        bu[u] = bit;
        lo[u] = ldu(pldb, o0);
        hi[u] = ldu(pldb, min(o0 + 4u, plast));
      }
#pragma unroll
      for (int u = 0; u < kD0Group; u++) {
        const uint32_t i = i0 + (uint32_t)u * kWaves;
        if (i >= npair) break;
        // a funnel shift of the two words the codes can span, then the two
        // fields (width 0 gives 0), then zigzag decoding of both halves
        const uint32_t w = wu[u];
        const uint32_t x = __builtin_amdgcn_alignbit(hi[u], lo[u], bu[u]);
        const uint32_t z = __builtin_amdgcn_ubfe(x, 0u, w) | (__builtin_amdgcn_ubfe(x, w, w) << 16);
        uint32_t q = ((z >> 1) & 0x7fff7fffu) ^ ((z & 0x00010001u) * 0xffffu);
        if (tileE) {
          // exact points take the marker in their half
          const uint32_t kc = min(2 * i + hf, ncw);
          const uint32_t e2 = (uint32_t)(cem[kc] >> (2 * lh)) & 3u;
          const uint32_t m = (e2 & 1u) * 0xffffu + (e2 & 2u) * 0x7fff8000u;
          q = (q & ~m) | (0x80008000u & m);
        }
        *reinterpret_cast<uint32_t *>(scs + 128 * i + 2 * (uint32_t)lane) = q;
      }
    }
  }
  __syncthreads();
  // codes by section index - J0
  const int16_t *const sc = scs + (J0 & 63u);

  D0Ctx t;
  t.sc = sc;
  t.cxo = cxo;
  t.cem = cem;
  t.xl = xl;
  t.xs = v.p + Xoff;
  t.J0 = J0;
  t.c0 = c0;
  t.xo0 = xo0;
  t.step = g.step;
  const char *__restrict__ sgb = reinterpret_cast<const char *>(sg);
  // output: the field (level 0) or the level's grid, from the block's first plane
  const uint32_t f1 = LV == 0 ? n1 : (uint32_t)D.gd[LV][1], f2 = LV == 0 ? n2 : (uint32_t)D.gd[LV][2];
  char *__restrict__ obase = reinterpret_cast<char *>((LV == 0 ? D.out : D.gp[LV]) + (size_t)(bp.o[0] / S) * f1 * f2);
  const bool zu = np == 2;
  const uint32_t rowB = f2 * 4u;
  const uint32_t xe0 = ((we * f1 + bp.o[1] / S) * f2 + bp.o[2] / S) * 4u;  // even plane, row 0
  const uint32_t xo0b = xe0 + f1 * f2 * 4u;                               // odd plane, row 0
  const uint32_t u = min((uint32_t)lane, mx - 1);                   // lanes past the row copy its last point
  const uint32_t lx0 = u >> 1;
  const bool xav = (u & 1u) && lx0 + 1 < gx;
  const uint32_t lg = lx0 * 4u, lx = u * 4u;
  constexpr uint32_t kRow = TD::Side * 4u, kPl = TD::Plane * 4u;
  const bool odd_u = (u & 1u) != 0;
  const uint32_t rown = all ? my : min(my, (owny + S - 1) / S);     // rows written

  // ---- even plane: rows v = 2a (odd u from codes, even u from level 1) and
  // v = 2a + 1 (every u from codes).  A wave reads the parents and codes of
  // kD0Rows rows, computes them, fixes any exact points, then stores.  Rows
  // past the block and lanes past a row work on a point inside the pair's
  // range (section indices clamped to [J0, J1)) and are not stored.
  const uint32_t jlast = J1 - 1;
  const uint32_t lxe = min(lx0, rowE > 0 ? rowE - 1 : 0u);   // an odd point of the row for even u
  // marching cubes' words: row (z, y) of the field, word o_x / 64 (points
  // u < min(mx, 64) of the row; u = 64 starts the next word)
  const uint64_t bnw = (uint64_t)D.bnw;
  const uint64_t wrow0 = ((uint64_t)(bp.o[0] + we) * n1 + bp.o[1]) * bnw + (bp.o[2] >> 6);
  const uint32_t nvb = min(mx, 64u);
  const unsigned long long vmask = __ballot((uint32_t)lane < nvb);
  const int nk = (LV == 0 && D.bits) ? D.nk : 0;
  // the store of a group's words: lane L holds row k = L mod 8 (its row in
  // the plane: rowof(k)) and isovalue 8 * set + L / 8
  auto bits_store = [&](const D0Bits &q, auto rowof) {
    const uint32_t k = (uint32_t)lane & 7u, jj = (uint32_t)lane >> 3;
    const uint32_t row = rowof(k);
#pragma unroll
    for (int set = 0; set < 2; set++) {
      const uint32_t j = jj + 8u * (uint32_t)set;
      if (8 * set < nk && j < (uint32_t)nk && row < rown)
        D.bits[(size_t)j * (size_t)D.bplane + wrow0 + (uint64_t)row * bnw] =
            ((unsigned long long)q.hi[set] << 32) | q.lo[set];
    }
  };
  // LDS code byte offsets: per lane, plus a uniform row part, clamped to the
  // pair's last point
  const char *__restrict__ scb = reinterpret_cast<const char *>(sc);
  const uint32_t cmax = 2 * (jlast - J0), ceb = 2 * lxe, cob = 2 * (rowE + u), cub = 2 * u;
  for (uint32_t a0 = wave; 2 * a0 < rown; a0 += kWaves * (kD0Rows / 2)) {
    float A0[kD0Rows / 2], A1[kD0Rows / 2], B0[kD0Rows / 2], B1[kD0Rows / 2];
    uint32_t je[kD0Rows / 2], jo[kD0Rows / 2];
    int32_t ze[kD0Rows / 2], zo[kD0Rows / 2];
#pragma unroll
    for (int k = 0; k < kD0Rows / 2; k++) {
      const uint32_t a = a0 + (uint32_t)k * kWaves;   // the row pair 2a, 2a + 1
      const uint32_t ga = min(a, gy - 1) * kRow + lg;
      A0[k] = d0_lds(sgb, ga);
      A1[k] = d0_lds(sgb, ga + 4);
      B0[k] = d0_lds(sgb, ga + kRow);
      B1[k] = d0_lds(sgb, ga + kRow + 4);
      je[k] = min(2 * a * RP + ceb, cmax);
      jo[k] = min(2 * a * RP + cob, cmax);
      ze[k] = *reinterpret_cast<const int16_t *>(scb + je[k]);
      zo[k] = *reinterpret_cast<const int16_t *>(scb + jo[k]);
    }
    float rv[kD0Rows];
#pragma unroll
    for (int k = 0; k < kD0Rows / 2; k++) {
      const uint32_t a = a0 + (uint32_t)k * kWaves;
      // v = 2a: a level-1 point (even u) or an x midpoint (odd u)
      const float A = d0_xavg(A0[k], A1[k], xav);
      rv[2 * k] = odd_u ? d0_quant(t, ze[k], A) : A0[k];
      // v = 2a + 1: midpoints along y of the x-averaged rows a, a + 1
      const float B = d0_xavg(B0[k], B1[k], xav);
      float pb = avg2(A, B);
      hold(pb);
      rv[2 * k + 1] = d0_quant(t, zo[k], a + 1 < gy ? pb : A);
    }
    if (tileE) {
      uint64_t anyE = 0;
#pragma unroll
      for (int k = 0; k < kD0Rows / 2; k++) anyE |= __ballot((odd_u && ze[k] == kD0ExactQ) || zo[k] == kD0ExactQ);
      if (anyE) {
#pragma unroll
        for (int k = 0; k < kD0Rows / 2; k++) {
          if (odd_u && ze[k] == kD0ExactQ) rv[2 * k] = d0_exact(t, J0 + je[k] / 2);
          if (zo[k] == kD0ExactQ) rv[2 * k + 1] = d0_exact(t, J0 + jo[k] / 2);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < kD0Rows / 2; k++) {
      const uint32_t a = a0 + (uint32_t)k * kWaves;
      if (2 * a < rown) stf(obase, xe0 + 2 * a * rowB + lx, rv[2 * k]);
      if (2 * a + 1 < rown) stf(obase, xe0 + (2 * a + 1) * rowB + lx, rv[2 * k + 1]);
    }
    if (nk) {
      D0Bits q{{0u, 0u}, {0u, 0u}};
      d0_bits_rows(D, q, rv, nk, vmask);
      // row k of the group: 2a + (k & 1), a = a0 + 4 (k / 2)
      bits_store(q, [&](uint32_t k) { return 2 * (a0 + (k >> 1) * kWaves) + (k & 1u); });
    }
  }
  // ---- odd plane: rows 2m (y even) and 2m + 1 (y odd), every u from codes
  if (has_odd && (all || (we + 1) * S < ownz)) {
    for (uint32_t m0 = wave; 2 * m0 < rown; m0 += kWaves * (kD0Rows / 2)) {
      float A0[kD0Rows / 2], A1[kD0Rows / 2], B0[kD0Rows / 2], B1[kD0Rows / 2];
      float C0[kD0Rows / 2], C1[kD0Rows / 2], E0[kD0Rows / 2], E1[kD0Rows / 2];
      uint32_t jc[kD0Rows / 2], jd[kD0Rows / 2];
      int32_t zc[kD0Rows / 2], zd[kD0Rows / 2];
#pragma unroll
      for (int k = 0; k < kD0Rows / 2; k++) {
        const uint32_t m = m0 + (uint32_t)k * kWaves;
        const uint32_t ga = min(m, gy - 1) * kRow + lg;
        A0[k] = d0_lds(sgb, ga);
        A1[k] = d0_lds(sgb, ga + 4);
        C0[k] = d0_lds(sgb, ga + kPl);
        C1[k] = d0_lds(sgb, ga + kPl + 4);
        B0[k] = d0_lds(sgb, ga + kRow);
        B1[k] = d0_lds(sgb, ga + kRow + 4);
        E0[k] = d0_lds(sgb, ga + kPl + kRow);
        E1[k] = d0_lds(sgb, ga + kPl + kRow + 4);
        jc[k] = min(2 * (s.Pe + 2 * m * mx) + cub, cmax);
        jd[k] = min(2 * (s.Pe + (2 * m + 1) * mx) + cub, cmax);
        zc[k] = *reinterpret_cast<const int16_t *>(scb + jc[k]);
        zd[k] = *reinterpret_cast<const int16_t *>(scb + jd[k]);
      }
      float rv[kD0Rows];
#pragma unroll
      for (int k = 0; k < kD0Rows / 2; k++) {
        const uint32_t m = m0 + (uint32_t)k * kWaves;
        const float A = d0_xavg(A0[k], A1[k], xav), Cc = d0_xavg(C0[k], C1[k], xav);
        float pc = avg2(A, Cc);
        hold(pc);
        rv[2 * k] = d0_quant(t, zc[k], zu ? pc : A);
        const bool yu = m + 1 < gy;
        const float B = d0_xavg(B0[k], B1[k], xav), Dd = d0_xavg(E0[k], E1[k], xav);
        float p0 = avg2(A, B), p1 = avg2(Cc, Dd);
        hold(p0);
        hold(p1);
        p0 = yu ? p0 : A;
        p1 = yu ? p1 : Cc;
        float pd = avg2(p0, p1);
        hold(pd);
        rv[2 * k + 1] = d0_quant(t, zd[k], zu ? pd : p0);
      }
      if (tileE) {
        uint64_t anyE = 0;
#pragma unroll
        for (int k = 0; k < kD0Rows / 2; k++) anyE |= __ballot(zc[k] == kD0ExactQ || zd[k] == kD0ExactQ);
        if (anyE) {
#pragma unroll
          for (int k = 0; k < kD0Rows / 2; k++) {
            if (zc[k] == kD0ExactQ) rv[2 * k] = d0_exact(t, J0 + jc[k] / 2);
            if (zd[k] == kD0ExactQ) rv[2 * k + 1] = d0_exact(t, J0 + jd[k] / 2);
          }
        }
      }
#pragma unroll
      for (int k = 0; k < kD0Rows / 2; k++) {
        const uint32_t m = m0 + (uint32_t)k * kWaves;
        if (2 * m < rown) stf(obase, xo0b + 2 * m * rowB + lx, rv[2 * k]);
        if (2 * m + 1 < rown) stf(obase, xo0b + (2 * m + 1) * rowB + lx, rv[2 * k + 1]);
      }
      if (nk) {
        D0Bits q{{0u, 0u}, {0u, 0u}};
        d0_bits_rows(D, q, rv, nk, vmask);
        // rows of the odd plane: n1 rows after the even plane's
        const uint32_t rbase = n1;
        auto rowof = [&](uint32_t k) { return 2 * (m0 + (k >> 1) * kWaves) + (k & 1u); };
        const uint32_t k = (uint32_t)lane & 7u, jj = (uint32_t)lane >> 3;
        const uint32_t row = rowof(k);
#pragma unroll
        for (int set = 0; set < 2; set++) {
          const uint32_t j = jj + 8u * (uint32_t)set;
          if (8 * set < nk && j < (uint32_t)nk && row < rown)
            D.bits[(size_t)j * (size_t)D.bplane + wrow0 + (uint64_t)(rbase + row) * bnw] =
                ((unsigned long long)q.hi[set] << 32) | q.lo[set];
        }
      }
    }
  }
  // ---- the points u = 64 (65-point rows), one row per lane, when the block
  // owns them (the last block along x) or writes its closed extent
  if constexpr (LV == 0) if (mx == 65 && (all || 64u < ownx)) {
    const uint32_t nrow = (has_odd && (all || we + 1 < ownz) ? 2u : 1u) * rown;
    for (uint32_t r0 = wave * 64; r0 < nrow; r0 += kWaves * 64) {
      const uint32_t rr = r0 + (uint32_t)lane;
      const uint32_t rc = min(rr, nrow - 1);
      const uint32_t w = rc >= rown ? 1u : 0u, vv = rc - w * rown;   // plane (0 even, 1 odd), row
      const uint32_t yl = vv >> 1;
      const bool yu = (vv & 1u) && yl + 1 < gy;
      const uint32_t yb = yu ? yl + 1 : yl;
      const float a0 = sg[yl * kD0Side + 32], b0 = sg[yb * kD0Side + 32];
      const float c0v = sg[kD0Plane + yl * kD0Side + 32], d0v = sg[kD0Plane + yb * kD0Side + 32];
      float r;
      if (w == 0 && !(vv & 1u)) {
        r = a0;  // a level-1 point
      } else {
        const float p0 = yu ? avg2(a0, b0) : a0;
        const float p1 = yu ? avg2(c0v, d0v) : c0v;
        const float p = (w == 1 && zu) ? avg2(p0, p1) : p0;
        const uint32_t j = min(w == 0 ? J0 + (vv >> 1) * RP + rowE + 64u : J0 + s.Pe + vv * mx + 64u, jlast);
        const int32_t q = sc[j - J0];
        r = q == kD0ExactQ ? d0_exact(t, j) : d0_quant(t, q, p);
      }
      if (rr < nrow) stf(obase, (w == 0 ? xe0 : xo0b) + vv * rowB + 256u, r);
      if (nk && rr < nrow) {
        // the field's last point along x: bit 0 of the row's next word, the
        // only point of that word
        const uint64_t widx = wrow0 + (w * n1 + vv) * bnw + 1;
        for (int j = 0; j < nk; j++) D.bits[(size_t)j * (size_t)D.bplane + widx] = r < D.kb[j] ? 1ull : 0ull;
      }
    }
  }
}

__global__ __launch_bounds__(kBS) void k_decode_l0t(DecPlan D) { decode_tile<0>(D); }
__global__ __launch_bounds__(kBS) void k_decode_l1t(DecPlan D) { decode_tile<1>(D); }

template <bool DIFF>
__global__ __launch_bounds__(kBS) void k_decode_l0(DecPlan D) { decode_fast<0, DIFF>(D); }
template <bool DIFF>
__global__ __launch_bounds__(kBS) void k_decode_l1(DecPlan D) { decode_fast<1, DIFF>(D); }
template <bool DIFF>
__global__ __launch_bounds__(kBS) void k_decode_l2(DecPlan D) { decode_fast<2, DIFF>(D); }

// Levels L .. 2 of a 64-cell block in one 1024-thread workgroup (the
// reconstruction half of k_encode_top).  The chunk headers of the levels'
// sections are read and checked (two waves per level, a tile each), every
// code is unpacked into LDS, then the threads' fixed 4-grid points are
// reconstructed level by level, coarsest first, predicting from the
// reconstruction in LDS, and the block's 4-grid is written to the level-2
// grid (every point of the closed extent; a neighbour writes the shared
// faces with the same values).
constexpr int kTopChunks = kTopCodes / 64;   // chunks of every level, each level 64-aligned

__global__ __launch_bounds__(kTopBS) void k_decode_top(DecPlan D) {
  __shared__ float R[kTopPts];
  __shared__ uint16_t sc[kTopCodes];
  __shared__ uint32_t cwb[kTopChunks], cwo[kTopChunks], cxo[kTopChunks];
  __shared__ unsigned long long cem[kTopChunks];
  __shared__ uint32_t base[kMaxLevels], npt[kMaxLevels];   // each level's first code and points
  __shared__ uint64_t spay[kMaxLevels], sxv[kMaxLevels];   // its payload and exact values (stream offsets)
  __shared__ uint32_t sbad;
  const uint32_t b = blockIdx.x;
  if (!block_needed(D, b)) return;
  const Geo &g = D.g;
  const int L = g.nL - 1;
  const BlockPos bp = block_pos(g, D.l0, b);
  const uint32_t wave = wave_index();
  const int lane = lane_id();
  const uint32_t d0 = ((bp.hi[0] - bp.o[0]) >> 2) + 1, d1 = ((bp.hi[1] - bp.o[1]) >> 2) + 1;
  const uint32_t d2 = ((bp.hi[2] - bp.o[2]) >> 2) + 1;
  uint32_t pc[kTopPer];
#pragma unroll
  for (int k = 0; k < kTopPer; k++) pc[k] = top_point(threadIdx.x + (uint32_t)k * kTopBS, d0, d1, d2, L);
  if (threadIdx.x == 0) {
    uint32_t off = 0;
    for (int l = L; l >= 2; l--) {
      const uint32_t n = sec_dims(bp, l, L).npts;
      base[l] = off;
      npt[l] = n;
      off += (n + 63) & ~63u;
    }
    sbad = 0u;
  }
  __syncthreads();
  // ---- chunk headers: wave 2 (L - l) + t reads tile t of level l's section
  {
    const int l = L - (int)(wave >> 1);
    const uint32_t t = wave & 1u;
    if (l >= 2) {
      const uint32_t nch = (npt[l] + 63) / 64;
      if (t * 64 < nch) {
        const SecView v = open_section(D, b, l, npt[l]);
        bool bad = !v.ok;
        if (v.ok) {
          if (t == 0 && lane == 0) {
            spay[l] = (uint64_t)(v.p - D.s) + v.Poff;
            sxv[l] = (uint64_t)(v.p - D.s) + v.Xoff;
          }
          const uint32_t c = t * 64 + (uint32_t)lane;
          const uint8_t *tt = v.p + 16 + 12 * (uint64_t)t;
          const uint32_t tw = ld32(tt), te = ld32(tt + 4), tx = ld32(tt + 8);
          const uint32_t hb = c < v.nch ? v.p[v.A + c] : 0u;
          const uint32_t w = hb & 31u, he = hb >> 7;
          const uint32_t wo = tw + wave_excl_sum_dpp(w), eo = te + wave_excl_sum_dpp(he);
          const bool badl = (w > (uint32_t)kMaxW) || (hb & 0x60u) || (wo + w > v.W) || (he && eo >= v.NE);
          const unsigned long long em = (he && !badl) ? ld64(v.p + v.Moff + 8 * (uint64_t)eo) : 0ull;
          const uint32_t pcnt = (uint32_t)__popcll(em);
          const uint32_t xo = tx + wave_excl_sum_dpp(pcnt);
          bad = __ballot(badl || xo + pcnt > v.NX) != 0ull;
          if (c < nch) {
            const uint32_t gi = base[l] / 64 + c;
            cwb[gi] = w;
            cwo[gi] = wo;
            cxo[gi] = xo;
            cem[gi] = em;
          }
        }
        if (bad && lane == 0) sbad = 1u;
      }
    }
  }
  __syncthreads();
  if (sbad) {
    if (threadIdx.x == 0) set_status(D, -4);
    return;
  }
  // ---- every code into LDS: wave w unpacks chunks w, w + 16, ... (its
  // level found from the levels' first chunks)
  {
    const uint32_t nct = base[2] / 64 + (npt[2] + 63) / 64;
    for (uint32_t gi = wave; gi < nct; gi += kTopWaves) {
      int l = L;
      while (l > 2 && gi >= base[l - 1] / 64) l--;
      const uint32_t w = (uint32_t)__builtin_amdgcn_readfirstlane(cwb[gi]);
      const uint32_t wo = (uint32_t)__builtin_amdgcn_readfirstlane(cwo[gi]);
      uint32_t zz = 0u;
      if (w) {
        const char *__restrict__ pay = reinterpret_cast<const char *>(D.s + spay[l]);
        const uint32_t bit = mul24s((uint32_t)lane, w), wi = bit >> 5;
        const uint32_t lo = ldu(pay, 8u * wo + 4u * wi), hi = ldu(pay, 8u * wo + 4u * min(wi + 1, 2 * w - 1));
        zz = __builtin_amdgcn_ubfe(__builtin_amdgcn_alignbit(hi, lo, bit), 0u, w);
      }
      sc[gi * 64 + (uint32_t)lane] = (uint16_t)zz;
    }
  }
  __syncthreads();
  // ---- the levels, coarsest first
  const float step = g.step;
  const bool lossless = g.lossless != 0;
  for (int l = L; l >= 2; l--) {
    const SecDims sd = sec_dims(bp, l, L);
    const uint32_t sh = (uint32_t)(l - 2), st = 1u << sh;     // the level's step on the 4-grid
    const uint32_t bl = base[l];
#pragma unroll
    for (int k = 0; k < kTopPer; k++) {
      if ((pc[k] >> 15) != (uint32_t)(l + 1)) continue;
      const uint32_t x = pc[k] & 31u, y = (pc[k] >> 5) & 31u, z = (pc[k] >> 10) & 31u;
      const uint32_t w = z >> sh, v = y >> sh, u = x >> sh;
      const uint32_t j = bl + sec_index(sd, l == L, w, v, u);
      const unsigned long long em = cem[j >> 6];
      float r;
      if ((em >> (j & 63u)) & 1ull) {
        const uint32_t xi = cxo[j >> 6] + (uint32_t)__popcll(em & ((1ull << (j & 63u)) - 1ull));
        r = __uint_as_float(ld32(D.s + sxv[l] + 4 * (uint64_t)xi));
      } else {
        float p = 0.0f;
        if (l < L) {
          // parents at -st and +st along the odd axes, the lower alone where
          // the upper is outside the domain
          const uint32_t oz = w & 1u, oy = v & 1u, ox = u & 1u;
          const uint32_t zl = z - oz * st, yl = y - oy * st, xl = x - ox * st;
          const bool zu = oz && z + st < d0, yu = oy && y + st < d1, xu = ox && x + st < d2;
          const uint32_t zb = zu ? z + st : zl, yb = yu ? y + st : yl, xb = xu ? x + st : xl;
          p = midpoint8(R[top_idx(zl, yl, xl)], R[top_idx(zl, yl, xb)], R[top_idx(zl, yb, xl)], R[top_idx(zl, yb, xb)],
                        R[top_idx(zb, yl, xl)], R[top_idx(zb, yl, xb)], R[top_idx(zb, yb, xl)], R[top_idx(zb, yb, xb)],
                        zu, yu, xu);
        }
        const uint32_t zc = sc[j];
        const int32_t q = (int32_t)(zc >> 1) ^ -(int32_t)(zc & 1u);
        r = lossless ? p : __fadd_rn(p, __fmul_rn((float)q, step));
      }
      R[top_idx(z, y, x)] = r;
    }
    __syncthreads();
  }
  // ---- the reconstructed 4-grid into the level-2 grid
  const uint32_t e1 = (uint32_t)D.gd[2][1], e2 = (uint32_t)D.gd[2][2];
  char *__restrict__ gb = reinterpret_cast<char *>(D.gp[2] + (((size_t)(bp.o[0] >> 2)) * e1 + (bp.o[1] >> 2)) * e2 +
                                                   (bp.o[2] >> 2));
#pragma unroll
  for (int k = 0; k < kTopPer; k++)
    if (pc[k] >> 15) {
      const uint32_t x = pc[k] & 31u, y = (pc[k] >> 5) & 31u, z = (pc[k] >> 10) & 31u;
      stf(gb, ((z * e1 + y) * e2 + x) * 4u, R[top_idx(z, y, x)]);
    }
}

// Even points of even rows in blocks one point wide along x (no level-0
// point in those rows writes them).
__global__ __launch_bounds__(kBS) void k_decode_thin(DecPlan D) {
  const Geo &g = D.g;
  const int64_t b = blockIdx.x;
  if (!block_needed(D, b)) return;
  int64_t o[3], hi[3];
  unit_ext(g, b, o, hi);
  if (hi[2] != o[2]) return;
  const int64_t cz = ((hi[0] - o[0]) >> 1) + 1, cy = ((hi[1] - o[1]) >> 1) + 1;
  for (int64_t i = threadIdx.x; i < cz * cy; i += kBS) {
    const int64_t z = o[0] + 2 * (i / cy), y = o[1] + 2 * (i % cy), x = o[2];
    D.out[(z * g.n[1] + y) * g.n[2] + x] = D.gp[1][((z >> 1) * D.gd[1][1] + (y >> 1)) * D.gd[1][2] + (x >> 1)];
  }
}

}  // namespace

// Blocks left out of a restricted reconstruction: their owned points (the
// closed extent minus the upper faces, which neighbours own) at the output
// level get one value on the same side of every requested isovalue as the
// whole block -- its min when min >= kmax (or the block is constant), else
// its max.  Runs before the decoders, whose closed-extent writes then
// restore the true values on faces shared with reconstructed blocks.
__global__ __launch_bounds__(kBS) void k_prune_fill(DecPlan D) {
  const Geo &g = D.g;
  const int64_t b = blockIdx.y;
  if (block_needed(D, b)) return;
  float mn, mx;
  block_range(D, b, mn, mx);
  const float c = (mn >= D.kmax || mn == mx) ? mn : mx;
  int64_t o[3], hi[3];
  unit_ext(g, b, o, hi);
  const int lo = D.lo;
  uint32_t lo3[3], hi3[3], dim[3];
  for (int a = 0; a < 3; a++) {
    const int64_t own = (hi[a] == g.n[a] - 1) ? g.n[a] : hi[a];  // exclusive end of the owned range
    lo3[a] = (uint32_t)(o[a] >> lo);
    hi3[a] = (uint32_t)((own + ((int64_t)1 << lo) - 1) >> lo);
    dim[a] = (uint32_t)(lo == 0 ? g.n[a] : D.gd[lo][a]);
  }
  float *out = lo == 0 ? D.out : D.gp[lo];
  const uint32_t cz = hi3[0] - lo3[0], cy = hi3[1] - lo3[1];
  const int wave = threadIdx.x / kWave;
  for (uint32_t r = blockIdx.x * kWaves + wave; r < cz * cy; r += gridDim.x * kWaves) {
    const uint32_t z = lo3[0] + r / cy, y = lo3[1] + r % cy;
    float *row = out + ((size_t)z * dim[1] + y) * dim[2];
    for (uint32_t x = lo3[2] + lane_id(); x < hi3[2]; x += kWave) row[x] = c;
  }
}

// Whether level 0 of this reconstruction runs by plane pairs (the kernel
// that also writes marching cubes' bits).
bool decode_tile0_used(const DecPlan &p) {
  const Geo &g = p.g;
  int64_t o[3], hi[3];
  largest_ext(g, o, hi);
  const bool slab32 = 4.0 * (double)(hi[0] - o[0] + 1) * (double)g.n[1] * (double)g.n[2] < 4294967296.0;
  return p.lo == 0 && p.tile0 && g.B == 64 && g.nL >= 2 && slab32 && p.l0.small && !g.diff && !g.lossless;
}

// Levels L .. 2 of 64-cell blocks in one workgroup per block (the output
// level 2 or finer).
static bool decode_top_used(const DecPlan &p) {
  const Geo &g = p.g;
  int64_t o[3], hi[3];
  largest_ext(g, o, hi);
  const bool slab32 = 4.0 * (double)(hi[0] - o[0] + 1) * (double)g.n[1] * (double)g.n[2] < 4294967296.0;
  return p.lo <= 2 && p.tile0 && g.B == 64 && g.nL >= 3 && slab32 && p.l0.small && !g.diff && !g.lossless;
}

// Level 1 likewise (as the output or on the way to level 0), below level 2.
static bool decode_tile1_used(const DecPlan &p) {
  const Geo &g = p.g;
  int64_t o[3], hi[3];
  largest_ext(g, o, hi);
  const bool slab32 = 4.0 * (double)(hi[0] - o[0] + 1) * (double)g.n[1] * (double)g.n[2] < 4294967296.0;
  return p.lo <= 1 && p.tile0 && g.B == 64 && g.nL >= 3 && slab32 && p.l0.small && !g.diff && !g.lossless;
}

void launch_decode(const DecPlan &p, hipStream_t s) {
  const Geo &g = p.g;
  const int L = g.nL - 1;
  int64_t o[3], hi[3];
  largest_ext(g, o, hi);
  if (p.prune) k_prune_fill<<<dim3(8, (unsigned)g.nblocks), dim3(kBS), 0, s>>>(p);
  const bool top = decode_top_used(p);
  if (top) {
    prof_mark("k_decode_coarse", s, 0);
    k_decode_top<<<dim3((unsigned)g.nblocks), dim3(kTopBS), 0, s>>>(p);
    prof_mark("k_decode_coarse", s, 1);
  } else if (L >= 3 && p.lo <= L) {
    prof_mark("k_decode_coarse", s, 0);
    k_decode_coarse<<<dim3((unsigned)g.nblocks), dim3(kBS), 0, s>>>(p);
    prof_mark("k_decode_coarse", s, 1);
  }
  // the specialized kernels address a block's slab with 32-bit offsets
  const bool slab32 = 4.0 * (double)(hi[0] - o[0] + 1) * (double)g.n[1] * (double)g.n[2] < 4294967296.0;
  for (int l = 2; l >= 1; l--) {
    if (l == 2 && top) continue;               // level 2 came with the coarser levels
    if (L >= l && p.lo <= l) {
      const Sec sl = sec_geom(o, hi, l, L);
      const int64_t ntl = ceil_div(ceil_div(sl.npts, 64), 64);
      const dim3 grid((unsigned)(ntl > 0 ? ntl : 1), (unsigned)g.nblocks);
      prof_mark(l == 1 ? "k_decode_l1" : "k_decode_l2", s, 0);
      if (l == 1 && decode_tile1_used(p)) {
        k_decode_l1t<<<dim3((unsigned)((g.B / 2 + 2) / 2), (unsigned)g.nblocks), dim3(kBS), 0, s>>>(p);
      } else if (l == 1 && L >= 2 && slab32 && p.l0.small) {
        // one tile per workgroup: 16 chunks per wave
        if (g.diff) k_decode_l1<true><<<grid, dim3(kBS), 0, s>>>(p);
        else k_decode_l1<false><<<grid, dim3(kBS), 0, s>>>(p);
      } else if (l == 2 && L >= 3 && slab32 && p.l0.small) {
        if (g.diff) k_decode_l2<true><<<grid, dim3(kBS), 0, s>>>(p);
        else k_decode_l2<false><<<grid, dim3(kBS), 0, s>>>(p);
      }
      else
        k_decode_level<<<grid, dim3(kBS), 0, s>>>(p, l);
      prof_mark(l == 1 ? "k_decode_l1" : "k_decode_l2", s, 1);
    }
  }
  if (p.lo == 0) {
    const Sec s0 = sec_geom(o, hi, 0, L);
    const int64_t ntile = ceil_div(ceil_div(s0.npts, 64), 64);
    prof_mark("k_decode_fine", s, 0);
    if (decode_tile0_used(p)) {
      k_decode_l0t<<<dim3((unsigned)((g.B + 2) / 2), (unsigned)g.nblocks), dim3(kBS), 0, s>>>(p);
    } else if (L >= 1 && slab32 && p.l0.small) {
      const int64_t nch0 = ceil_div(s0.npts, 64);
      const int64_t gx0 = ceil_div(nch0 > 0 ? nch0 : 1, (int64_t)kWaves * p.cpw0);
      if (g.diff) k_decode_l0<true><<<dim3((unsigned)gx0, (unsigned)g.nblocks), dim3(kBS), 0, s>>>(p);
      else k_decode_l0<false><<<dim3((unsigned)gx0, (unsigned)g.nblocks), dim3(kBS), 0, s>>>(p);
    } else {
      k_decode_fine<<<dim3((unsigned)ceil_div(ntile > 0 ? ntile : 1, kWaves), (unsigned)g.nblocks), dim3(kBS), 0, s>>>(p);
    }
    prof_mark("k_decode_fine", s, 1);
    if (L >= 1 && g.n[2] == 1) {   // only a field one point wide along x has blocks that wide
      prof_mark("k_decode_thin", s, 0);
      k_decode_thin<<<dim3((unsigned)g.nblocks), dim3(kBS), 0, s>>>(p);
      prof_mark("k_decode_thin", s, 1);
    }
  }
}

__global__ void k_status_reset(int32_t *status) {
  if (threadIdx.x == 0) *status = 0;
}

void launch_status_reset(int32_t *status, hipStream_t s) { k_status_reset<<<dim3(1), dim3(64), 0, s>>>(status); }

}  // namespace chr
