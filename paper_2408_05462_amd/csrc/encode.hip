// encode.hip -- CHR compression kernels for gfx950.
//
// One 64-lane wave encodes one 64-point chunk of a (block, level) section:
// every lane predicts its point from the reconstructed coarser grid,
// quantizes, checks the error bound, checks that the point stays on the same
// side of every candidate isovalue (Sec. II.B: topology preservation) and, if
// either check fails, stores the point exactly.  The chunk's zigzag codes are
// bit-packed at the wave's maximum width through LDS, exact points are
// compacted with a ballot and mbcnt.  Statistics (block min/max, counts) are
// reduced per workgroup into a record of their own -- no atomics -- and
// folded per block and per stream by the table and header kernels.
//
// Launch sequence: coarse levels (one workgroup per block, levels nL-1..1,
// each level's compact grid written before the next level reads it) ->
// level 0 (a 2D grid over chunk groups x blocks) -> scan of the per-chunk
// sizes -> section sizes -> scan of section sizes -> section headers and
// tables -> chunk copy into the stream -> block table -> stream header.
#include "chr_plan.h"

namespace chr {
namespace {

constexpr int kBS = 256;
constexpr int kWaves = kBS / kWave;
constexpr int kChunksPerWave = 4;
constexpr int kChunksPerWG = kWaves * kChunksPerWave;

// Multilinear midpoint prediction of point (z,y,x) of level l from the
// compact grid Gp of level l+1 (dims g0 x g1 x g2): along each axis where the
// coordinate is an odd multiple of 2^l the two parents at -2^l and +2^l are
// averaged (the lower one alone if the upper one is outside the domain);
// averages along x first, then y, then z.
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

// Carries the block's points of the coarser compact grid (dims sd, shift sh
// from full resolution) over to the even positions of the finer one (dims
// dd): one row per wave step, starting at wave `first`, stepping by `step`.
__device__ inline void copy_coarse(const float *__restrict__ src, const int64_t *sd, float *__restrict__ dst,
                                   const int64_t *dd, const int64_t o[3], const int64_t hi[3], int sh,
                                   uint32_t first, uint32_t step) {
  const uint32_t c0 = (uint32_t)((hi[0] - o[0]) >> sh) + 1, c1 = (uint32_t)((hi[1] - o[1]) >> sh) + 1;
  const uint32_t c2 = (uint32_t)((hi[2] - o[2]) >> sh) + 1;
  const uint32_t zo = (uint32_t)(o[0] >> sh), yo = (uint32_t)(o[1] >> sh), xo = (uint32_t)(o[2] >> sh);
  const uint32_t s1 = (uint32_t)sd[1], s2 = (uint32_t)sd[2], d1 = (uint32_t)dd[1], d2 = (uint32_t)dd[2];
  for (uint32_t r = first; r < c0 * c1; r += step) {
    const uint32_t w = r / c1, v = r - w * c1;
    const size_t srow = ((size_t)(zo + w) * s1 + (yo + v)) * s2 + xo;
    const size_t drow = ((size_t)(2 * (zo + w)) * d1 + 2 * (yo + v)) * d2 + 2 * xo;
    for (uint32_t u = lane_id(); u < c2; u += kWave) dst[drow + 2 * u] = src[srow + u];
  }
}

// Error-bounded linear quantization: q = rint((x-p)/(2e)) (half even), the
// reconstruction p + q*2e, an outlier when |q| > qmax or the reconstruction
// misses the bound (checked in double).  Lossless mode: q = 0, x' = p.
__device__ inline void quantize(const QuantP &g, int qmax, float x, float p, int32_t &q, int &O, float &xr) {
  if (g.lossless) {
    q = 0;
    xr = p;
    O = __float_as_uint(p) != __float_as_uint(x);
    return;
  }
  const float d = __fsub_rn(x, p);
  const float qf = rintf(__fmul_rn(d, g.inv));
  if (!(fabsf(qf) <= (float)qmax)) {
    q = 0; O = 1; xr = p;
    return;
  }
  xr = __fadd_rn(p, __fmul_rn(qf, g.step));
  q = (int32_t)qf;
  O = !(fabs((double)xr - (double)x) <= g.e);
}

__device__ inline void quantize(const Geo &g, float x, float p, int32_t &q, int &O, float &xr) {
  quantize(quant_pick(g, false), g.qmax, x, p, q, O, xr);
}

// Number of candidate isovalues k with k <= v; equal counts for x and x'
// mean x' lies on the same side of every candidate as x.
// KB is a compile-time bound on the number of candidates (K <= KB), so
// the loop is fully unrolled with constant indices.
template <int KB>
__device__ inline int rank_of(const float (&iso)[KB], int K, float v) {
  int r = 0;
#pragma unroll
  for (int j = 0; j < KB; j++)
    if (j < K) r += (iso[j] <= v) ? 1 : 0;
  return r;
}

__device__ inline void part_init(Part &a) {
  a.rmin = a.xmin = 0xffffffffu;
  a.rmax = a.xmax = 0u;
  a.nonfinite = a.nO = a.nC = a.pad = 0;
}

// Reduces the threads' records of one workgroup and stores it at *dst.
__device__ void part_store(const Part &a, Part *dst) {
  __shared__ Part red[kWaves];
  Part r;
  r.rmin = wave_min_dpp(a.rmin); r.rmax = wave_max_dpp(a.rmax);
  r.xmin = wave_min_dpp(a.xmin); r.xmax = wave_max_dpp(a.xmax);
  r.nonfinite = wave_or_dpp(a.nonfinite); r.nO = wave_sum_dpp(a.nO); r.nC = wave_sum_dpp(a.nC);
  r.pad = 0;
  if (lane_id() == 0) red[threadIdx.x / kWave] = r;
  __syncthreads();
  if (threadIdx.x == 0) {
    Part t = red[0];
    for (int i = 1; i < kWaves; i++) {
      t.rmin = min(t.rmin, red[i].rmin); t.rmax = max(t.rmax, red[i].rmax);
      t.xmin = min(t.xmin, red[i].xmin); t.xmax = max(t.xmax, red[i].xmax);
      t.nonfinite |= red[i].nonfinite; t.nO += red[i].nO; t.nC += red[i].nC;
    }
    *dst = t;
  }
}

// Encodes chunk c of the level-l section of block b into its slot.
template <int KB>
__device__ void enc_chunk(const EncPlan &P, int l, int64_t b, const int64_t o[3], const int64_t own[3],
                          const NearSel &ns, const Sec &s, uint32_t c, uint32_t *pack, Part &acc) {
  const Geo &g = P.g;
  float iso[KB];
#pragma unroll
  for (int jj = 0; jj < KB; jj++) iso[jj] = g.iso[jj];
  const int L = g.nL - 1;
  const int lane = lane_id();
  const uint32_t j = c * kWave + (uint32_t)lane;
  const bool valid = j < s.npts;
  float x = 0.f, xr = 0.f;
  int32_t q = 0;
  int O = 0, C = 0;
  if (valid) {
    uint32_t w, v, u;
    sec_point(s, j, w, v, u);
    const uint32_t z = (uint32_t)o[0] + (w << l), y = (uint32_t)o[1] + (v << l), xx = (uint32_t)o[2] + (u << l);
    const size_t gi = ((size_t)z * (uint32_t)g.n[1] + y) * (uint32_t)g.n[2] + xx;
    x = P.x[gi];
    float p = 0.0f;
    if (l < L) {
      const int64_t *gd = P.gd[l + 1];
      p = predict(P.G + P.g_off[l + 1], (uint32_t)gd[0], (uint32_t)gd[1], (uint32_t)gd[2], l, z, y, xx);
    }
    quantize(quant_pick(g, g.diff && !near_at(ns, z, y, xx)), g.qmax, x, p, q, O, xr);
    if (!O && g.K > 0) C = rank_of<KB>(iso, g.K, x) != rank_of<KB>(iso, g.K, xr);
    if (O || C) { xr = x; q = 0; }
    if (l >= 1) {
      const int64_t *gd = P.gd[l];
      P.G[P.g_off[l] + ((size_t)(z >> l) * (uint32_t)gd[1] + (y >> l)) * (uint32_t)gd[2] + (xx >> l)] = xr;
    }
    const uint32_t ro = ord_of(xr), xo = ord_of(x);
    acc.rmin = min(acc.rmin, ro); acc.rmax = max(acc.rmax, ro);
    acc.xmin = min(acc.xmin, xo); acc.xmax = max(acc.xmax, xo);
    acc.nonfinite |= !isfinite(x);
    if (z < own[0] && y < own[1] && xx < own[2]) { acc.nO += O; acc.nC += C; }
    if (P.codes) P.codes[gi] = q;
    if (P.flags) P.flags[gi] = (uint8_t)(O | (C << 1));
  }
  const bool E = valid && (O || C);
  const uint32_t zz = (valid && !E) ? (((uint32_t)q << 1) ^ (uint32_t)(q >> 31)) : 0u;
  const uint32_t orv = wave_or_dpp(zz);
  const int wb = orv ? 32 - __clz((int)orv) : 0;
  const unsigned long long em = __ballot(E);
  const int64_t slot = slot_of(P, l, b) + c;

  // pack the codes at bit lane*wb through LDS
  if (lane < 32) pack[lane] = 0u;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  if (wb && zz) {
    const uint32_t bit = (uint32_t)lane * (uint32_t)wb, wi = bit >> 5, off = bit & 31u;
    __hip_atomic_fetch_or(&pack[wi], zz << off, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    if (off + (uint32_t)wb > 32u)
      __hip_atomic_fetch_or(&pack[wi + 1], zz >> (32u - off), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
  if (lane < 2 * wb) P.pay[slot * 32 + lane] = pack[lane];
  if (E) P.exv[slot * 64 + lanes_below(em)] = x;
  if (lane == 0) {
    P.cnt[slot] = U4{(uint32_t)wb, em ? 1u : 0u, (uint32_t)__popcll(em), 0u};
    if (em) P.emask[slot] = em;
  }
  __builtin_amdgcn_wave_barrier();
}

// Zero counts for a slot past the section (the uniform layout's padding;
// merged units have no padding slots).
__device__ inline void zero_slot(const EncPlan &P, int l, int64_t b, uint32_t c) {
  if (P.ubase) return;
  if (lane_id() == 0) P.cnt[slot_of(P, l, b) + c] = U4{0, 0, 0, 0};
}

// First coordinate past the points a unit owns along each axis: the upper
// face belongs to the next unit unless it is the domain's last plane.
__device__ inline void owned_end(const Geo &g, const int64_t hi[3], int64_t own[3]) {
  for (int a = 0; a < 3; a++) own[a] = (hi[a] < g.n[a] - 1) ? hi[a] : g.n[a];
}

// Levels nL-1 .. 2 of one block per workgroup.
template <int KB>
__global__ __launch_bounds__(kBS) void k_encode_coarse(EncPlan P, int lmin) {
  __shared__ uint32_t pack[kWaves][32];
  const Geo &g = P.g;
  const int L = g.nL - 1;
  const int64_t b = blockIdx.x;
  const int wave = threadIdx.x / kWave;
  int64_t o[3], hi[3], own[3];
  unit_ext(g, b, o, hi);
  owned_end(g, hi, own);
  const NearSel ns = g.diff ? near_sel(g, P.act, 1u, b, o, hi) : NearSel{};
  Part acc;
  part_init(acc);
  for (int l = L; l >= lmin; l--) {
    if (l < L) {
      // the block's points of the coarser grid carry over unchanged
      const int sh = l + 1;
      copy_coarse(P.G + P.g_off[l + 1], P.gd[l + 1], P.G + P.g_off[l], P.gd[l], o, hi, sh, wave, kWaves);
    }
    const Sec s = sec_geom(o, hi, l, L);
    const uint32_t nch = (s.npts + 63) / 64;
    for (uint32_t c = wave; c < P.maxch[l]; c += kWaves) {
      if (c < nch) enc_chunk<KB>(P, l, b, o, own, ns, s, c, pack[wave], acc);
      else zero_slot(P, l, b, c);
    }
    __syncthreads();
  }
  part_store(acc, &P.part[b * P.part_per_block + (P.part_per_block - 1)]);
}

// Level 1 over (chunk groups, blocks); the block's level-2 points are
// copied into the level-1 grid by the same workgroups.
template <int KB>
__global__ __launch_bounds__(kBS) void k_encode_l1(EncPlan P) {
  __shared__ uint32_t pack[kWaves][32];
  const Geo &g = P.g;
  const int L = g.nL - 1;
  uint32_t bx, by;
  xcd_remap(bx, by);
  const int64_t b = by;
  const int wave = threadIdx.x / kWave;
  int64_t o[3], hi[3], own[3];
  unit_ext(g, b, o, hi);
  owned_end(g, hi, own);
  const NearSel ns = g.diff ? near_sel(g, P.act, 1u, b, o, hi) : NearSel{};
  if (L >= 2) {
    copy_coarse(P.G + P.g_off[2], P.gd[2], P.G + P.g_off[1], P.gd[1], o, hi, 2, bx * kWaves + wave,
                gridDim.x * kWaves);
  }
  const Sec s = sec_geom(o, hi, 1, L);
  const uint32_t nch = (s.npts + 63) / 64;
  Part acc;
  part_init(acc);
  for (int k = 0; k < kChunksPerWave; k++) {
    const uint32_t c = (bx * kChunksPerWave + k) * kWaves + wave;
    if (c >= P.maxch[1]) break;
    if (c < nch) enc_chunk<KB>(P, 1, b, o, own, ns, s, c, pack[wave], acc);
    else zero_slot(P, 1, b, c);
  }
  part_store(acc, &P.part[b * P.part_per_block + P.part_l1 + bx]);
}

// Level 0: a 2D grid of (chunk groups, blocks).
template <int KB>
__global__ __launch_bounds__(kBS) void k_encode_fine(EncPlan P) {
  __shared__ uint32_t pack[kWaves][32];
  const Geo &g = P.g;
  const int L = g.nL - 1;
  const int64_t b = blockIdx.y;
  const int wave = threadIdx.x / kWave;
  int64_t o[3], hi[3], own[3];
  unit_ext(g, b, o, hi);
  owned_end(g, hi, own);
  const NearSel ns = g.diff ? near_sel(g, P.act, 1u, b, o, hi) : NearSel{};
  const Sec s = sec_geom(o, hi, 0, L);
  const uint32_t nch = (s.npts + 63) / 64;
  Part acc;
  part_init(acc);
  for (int k = 0; k < P.cpw0; k++) {
    const uint32_t c = (blockIdx.x * P.cpw0 + k) * kWaves + wave;
    if (c >= P.maxch[0]) break;
    if (c < nch) enc_chunk<KB>(P, 0, b, o, own, ns, s, c, pack[wave], acc);
    else zero_slot(P, 0, b, c);
  }
  part_store(acc, &P.part[b * P.part_per_block + blockIdx.x]);
}

// Packs the chunk of this wave (codes zz, exact flags E, exact values x) into
// slot `slot`.
__device__ inline void pack_chunk(const EncPlan &P, int64_t slot, uint32_t zz, bool E, float x, uint32_t *pack) {
  const int lane = lane_id();
  const uint32_t orv = wave_or_dpp(zz);
  const int wb = orv ? 32 - __clz((int)orv) : 0;
  const unsigned long long em = __ballot(E);
  if (lane < 32) pack[lane] = 0u;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  if (zz) {
    const uint32_t bit = (uint32_t)lane * (uint32_t)wb, wi = bit >> 5, off = bit & 31u;
    __hip_atomic_fetch_or(&pack[wi], zz << off, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    if (off + (uint32_t)wb > 32u)
      __hip_atomic_fetch_or(&pack[wi + 1], zz >> (32u - off), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
  if (lane < 2 * wb) P.pay[slot * 32 + lane] = pack[lane];
  if (E) P.exv[slot * 64 + lanes_below(em)] = x;
  if (lane == 0) {
    P.cnt[slot] = U4{(uint32_t)wb, em ? 1u : 0u, (uint32_t)__popcll(em), 0u};
    if (em) P.emask[slot] = em;
  }
  __builtin_amdgcn_wave_barrier();
}

// Levels 0, 1 and 2 below a coarser level (level LV + 1 exists): the
// arithmetic of enc_chunk with the level fixed, for block shapes whose index
// products fit 24 bits (the host table's reciprocals divide the section
// index; 32-bit byte offsets from uniform bases: the block's first plane of
// the field, of the parent grid LV + 1 and, above level 0, of grid LV, which
// it fills).  A wave handles CPW chunks (P.cpw0 at level 0, kChunksPerWave
// above), G at a time: the loads of all G are issued first, every value is
// computed before any branch or store, so a wave keeps several chunks' reads
// in flight and no load is left pending on a path.  The optional per-point
// outputs, and the per-point choice of quantizer of differentiated error
// control, are compiled in only when requested.
template <int LV, bool AUX, int KB, int G, bool DIFF>
__device__ __forceinline__ void encode_fast(const EncPlan &P, uint32_t (*pack)[32]) {
  uint32_t gxi, b;
  xcd_remap(gxi, b);
  const uint32_t wave = wave_index();
  const int lane = lane_id();
  // Every uniform value the loop needs is copied into a local first, so it
  // stays in scalar registers across the loop's stores.
  const Geo &gq = P.g;
  const BlockPos bp = block_pos(gq, P.l0, b);
  NearSel ns{};
  bool mixed = false, allfar = false;
  if (DIFF) {
    const int64_t o[3] = {bp.o[0], bp.o[1], bp.o[2]}, hi[3] = {bp.hi[0], bp.hi[1], bp.hi[2]};
    ns = near_sel(gq, P.act, 1u, b, o, hi);
    mixed = ns.lut != 0u && ns.lut != kNearAll;   // else one quantizer for the whole block
    allfar = ns.lut == 0u;
  }
  const QuantP qblk = quant_pick(gq, allfar);     // scalar constants of an unmixed block
  if (LV >= 1) {
    // the block's points of grid LV + 1 carry over into grid LV unchanged
    const int64_t o[3] = {bp.o[0], bp.o[1], bp.o[2]}, hi[3] = {bp.hi[0], bp.hi[1], bp.hi[2]};
    copy_coarse(P.G + P.g_off[LV + 1], P.gd[LV + 1], P.G + P.g_off[LV], P.gd[LV], o, hi, LV + 1,
                gxi * kWaves + wave, gridDim.x * kWaves);
  }
  const Sec s = LV == 0 ? P.l0.sec[bp.cls] : LV == 1 ? P.l0.sec1[bp.cls] : P.l0.sec2[bp.cls];
  const SecR rc = LV == 0 ? P.l0.rc[bp.cls] : LV == 1 ? P.l0.rc1[bp.cls] : P.l0.rc2[bp.cls];
  const uint32_t nch = (s.npts + 63) / 64;
  const uint32_t maxch = (uint32_t)P.maxch[LV];
  const uint32_t n1 = (uint32_t)gq.n[1], n2 = (uint32_t)gq.n[2];
  // block origin on the level-LV grid (y, x) and the parent grid's slab
  const uint32_t oyl = bp.o[1] >> LV, oxl = bp.o[2] >> LV;
  const uint32_t h0 = (uint32_t)P.gd[LV + 1][0], h1 = (uint32_t)P.gd[LV + 1][1], h2 = (uint32_t)P.gd[LV + 1][2];
  const uint32_t zp = bp.o[0] >> (LV + 1);
  const uint32_t f1 = (uint32_t)P.gd[LV][1], f2 = (uint32_t)P.gd[LV][2];  // grid LV (filled for LV >= 1)
  // uniform bases; the launcher guarantees the block's slab spans < 4 GiB
  const char *__restrict__ xbase = reinterpret_cast<const char *>(P.x + (size_t)bp.o[0] * n1 * n2);
  const char *__restrict__ Pb = reinterpret_cast<const char *>(P.G + P.g_off[LV + 1] + (size_t)zp * h1 * h2);
  char *__restrict__ GLb = reinterpret_cast<char *>(P.G + P.g_off[LV] + (size_t)(bp.o[0] >> LV) * f1 * f2);
  const uint32_t h2x4 = h2 * 4u, h12x4 = h1 * h2 * 4u;
  const uint32_t ownz = bp.own[0] - bp.o[0], owny = bp.own[1], ownx = bp.own[2];
  const int64_t slot0 = P.slot_base[LV] + (int64_t)b * maxch;
  U4 *__restrict__ cnt = P.cnt;
  uint32_t *__restrict__ pay = P.pay;
  unsigned long long *__restrict__ emask = P.emask;
  float *__restrict__ exv = P.exv;
  int32_t *codes = P.codes;
  uint8_t *flags = P.flags;
  const int K = gq.K;
  float iso[KB];
#pragma unroll
  for (int jj = 0; jj < KB; jj++) iso[jj] = gq.iso[jj];
  Part acc;
  part_init(acc);
  const int cpw = LV == 0 ? P.cpw0 : kChunksPerWave;
  const uint32_t jmax = s.npts ? s.npts - 1 : 0u;
  // lanes past the section (and chunks past it) read a clamped point and
  // discard it
#pragma unroll 1
  for (int k0 = 0; k0 < cpw; k0 += G) {
    float xs[G], pa[G][8], xrs[G];
    bool zu[G], yu[G], xu[G], in[G], own[G], far[G];
    uint32_t gi[G], go[G];
#pragma unroll
    for (int u = 0; u < G; u++) {
      const uint32_t c = (gxi * cpw + k0 + u) * kWaves + wave;
      const uint32_t jr = c * kWave + (uint32_t)lane;
      uint32_t w, v, uu;
      sec_point24(s, rc, min(jr, jmax), w, v, uu);
      // (w, V, U): the point on the level-LV grid (w relative to the block)
      const uint32_t V = oyl + v, U = oxl + uu;
      const uint32_t zr = w << LV, y = V << LV, xx = U << LV;
      const uint32_t prow = mad24s(zr, n1, y);
      xs[u] = ldf(xbase, mad24s(prow, n2, xx) * 4u);
      const uint32_t zl = w >> 1, yl = V >> 1, xl = U >> 1;
      zu[u] = (w & 1u) && (zp + zl + 1 < h0);
      yu[u] = (V & 1u) && (yl + 1 < h1);
      xu[u] = (U & 1u) && (xl + 1 < h2);
      // byte offsets of the eight parents in the block's slab of grid LV + 1
      const uint32_t o00 = mad24s(mad24s(zl, h1, yl), h2, xl) * 4u;
      const uint32_t dxo = xu[u] ? 4u : 0u, dyo = yu[u] ? h2x4 : 0u, dzo = zu[u] ? h12x4 : 0u;
      const uint32_t o01 = o00 + dyo, o10 = o00 + dzo, o11 = o10 + dyo;
      pa[u][0] = ldf(Pb, o00); pa[u][1] = ldf(Pb, o00 + dxo);
      pa[u][2] = ldf(Pb, o01); pa[u][3] = ldf(Pb, o01 + dxo);
      pa[u][4] = ldf(Pb, o10); pa[u][5] = ldf(Pb, o10 + dxo);
      pa[u][6] = ldf(Pb, o11); pa[u][7] = ldf(Pb, o11 + dxo);
      in[u] = jr < s.npts;
      own[u] = zr < ownz && y < owny && xx < ownx;
      far[u] = DIFF && mixed && !near_at(ns, bp.o[0] + zr, y, xx);
      gi[u] = AUX ? mad24s(prow, n2, xx) : 0u;                  // the point in the block's slab
      go[u] = LV >= 1 ? mad24s(mad24s(w, f1, V), f2, U) * 4u : 0u;  // its slot in grid LV
    }
    // every point's arithmetic before any branch, so every load is consumed
    // on every path (lanes past the section compute on their clamped point
    // and are masked)
    uint32_t zzs[G];
    bool Es[G];
#pragma unroll
    for (int u = 0; u < G; u++) {
      const float x = xs[u];
      const float p = midpoint8(pa[u][0], pa[u][1], pa[u][2], pa[u][3], pa[u][4], pa[u][5], pa[u][6], pa[u][7],
                                zu[u], yu[u], xu[u]);
      int32_t q;
      int O, C = 0;
      float xr;
      if (DIFF && mixed) quantize(quant_pick(gq, far[u]), gq.qmax, x, p, q, O, xr);
      else if (DIFF) quantize(qblk, gq.qmax, x, p, q, O, xr);
      else quantize(gq, x, p, q, O, xr);
      if (!O && K > 0) C = rank_of<KB>(iso, K, x) != rank_of<KB>(iso, K, xr);
      if (O || C) { xr = x; q = 0; }
      zzs[u] = in[u] ? (((uint32_t)q << 1) ^ (uint32_t)(q >> 31)) : 0u;
      Es[u] = in[u] && (O || C);
      xrs[u] = xr;
      if (in[u]) {
        const uint32_t ro = ord_of(xr), xo = ord_of(x);
        acc.rmin = min(acc.rmin, ro); acc.rmax = max(acc.rmax, ro);
        acc.xmin = min(acc.xmin, xo); acc.xmax = max(acc.xmax, xo);
        acc.nonfinite |= !isfinite(x);
        if (own[u]) { acc.nO += O; acc.nC += C; }
        if (AUX) {
          const size_t gidx = (size_t)bp.o[0] * n1 * n2 + gi[u];
          if (codes) codes[gidx] = q;
          if (flags) flags[gidx] = (uint8_t)(O | (C << 1));
        }
      }
      hold(zzs[u]);
      hold(xrs[u]);
    }
#pragma unroll
    for (int u = 0; u < G; u++) {
      const uint32_t c = (gxi * cpw + k0 + u) * kWaves + wave;
      if (c >= maxch) break;
      const int64_t slot = slot0 + c;
      if (c >= nch) {
        if (lane == 0) cnt[slot] = U4{0, 0, 0, 0};
        continue;
      }
      // levels >= 1: the reconstructed value is a parent of the next level
      if (LV >= 1 && in[u]) stf(GLb, go[u], xrs[u]);
      const float x = xs[u];
      const uint32_t zz = zzs[u];
      const bool E = Es[u];
      // pack the codes at bit lane*wb through LDS
      uint32_t *pk = pack[wave];
      const uint32_t orv = wave_or_dpp(zz);
      const int wb = orv ? 32 - __clz((int)orv) : 0;
      const unsigned long long em = __ballot(E);
      if (lane < 32) pk[lane] = 0u;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      if (zz) {
        const uint32_t bit = (uint32_t)lane * (uint32_t)wb, wi = bit >> 5, off = bit & 31u;
        __hip_atomic_fetch_or(&pk[wi], zz << off, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        if (off + (uint32_t)wb > 32u)
          __hip_atomic_fetch_or(&pk[wi + 1], zz >> (32u - off), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
      if (lane < 2 * wb) pay[slot * 32 + lane] = pk[lane];
      if (E) exv[slot * 64 + lanes_below(em)] = x;
      if (lane == 0) {
        cnt[slot] = U4{(uint32_t)wb, em ? 1u : 0u, (uint32_t)__popcll(em), 0u};
        if (em) emask[slot] = em;
      }
      __builtin_amdgcn_wave_barrier();
    }
  }
  part_store(acc, &P.part[(int64_t)b * P.part_per_block + (LV == 0 ? 0 : LV == 1 ? P.part_l1 : P.part_l2) + gxi]);
}

template <bool AUX, int KB, int G, bool DIFF>
__global__ __launch_bounds__(kBS) __attribute__((amdgpu_waves_per_eu(DIFF ? 6 : 1))) void k_encode_l0(EncPlan P) {
  __shared__ uint32_t pack[kWaves][32];
  encode_fast<0, AUX, KB, G, DIFF>(P, pack);
}

template <bool AUX, int KB, int G, bool DIFF>
__global__ __launch_bounds__(kBS) __attribute__((amdgpu_waves_per_eu(DIFF ? 6 : 1))) void k_encode_l1s(EncPlan P) {
  __shared__ uint32_t pack[kWaves][32];
  encode_fast<1, AUX, KB, G, DIFF>(P, pack);
}

template <bool AUX, int KB, int G, bool DIFF>
__global__ __launch_bounds__(kBS) __attribute__((amdgpu_waves_per_eu(DIFF ? 6 : 1))) void k_encode_l2s(EncPlan P) {
  __shared__ uint32_t pack[kWaves][32];
  encode_fast<2, AUX, KB, G, DIFF>(P, pack);
}

// ------------------------------------------------------- level 0 by plane pairs
//
// Level 0 of 64-cell blocks (at most 65 points per axis) below a coarser
// level, one workgroup per (pair of z-planes, block).  The workgroup stages
// the two planes of the level-1 grid that hold its points' parents in LDS,
// then predicts and quantizes its points row by row along x (lane = point),
// so a row's parity pattern, its parent rows and its section offset are
// wave-uniform, and scatters each code into LDS at its position in the
// section (the section is lexicographic over the level-0 points of the
// closed block, so a row's points are consecutive there).  The waves then
// pack whole 64-point chunks from LDS into their slots.  A chunk that starts
// in this pair and ends in the next one is finished here: its last points
// (the first ones of the next even plane) are computed as well and the next
// workgroup, which computes them again, leaves that chunk alone.
//
// Row kinds of a pair (w = 2*w2 even, w + 1 odd; v = row, u = x index):
//   A: even plane, even rows -- only odd u are level-0 points; two rows per
//      wave (lanes 0-31: row v, 32-63: row v + 2);
//   F: every other row (even plane odd rows, all odd-plane rows) -- every u,
//      u = lane for u < 64;
//   C: the points u = 64 of the F rows, one row per lane;
//   S: the points of the chunk tail in the next plane pair.

constexpr int kT0Side = 33;                  // level-1 points per axis of a 64-cell block
constexpr int kT0Plane = 1152;               // staged plane stride (floats): 33 rows of 33, a byte offset that
                                             // fits an LDS instruction's immediate
constexpr int kT0Codes = 7361 + 63;          // most section points of a pair, plus a chunk's tail
constexpr int kT0Spare = 64;                 // LDS codes before the tile's first chunk (at most 63 used)
constexpr int kT0Group = 8;                  // rows whose loads a wave issues together
constexpr uint16_t kT0Exact = 0xffffu;       // LDS code of a point stored exactly (codes are < 2^16 - 1)

// Per-tile state of the finishing steps: LDS codes (indexed by section
// position: `sc` is offset so that the points of the previous pair's last
// chunk, at most 63 before the tile's first chunk, land in a spare prefix),
// the slots' exact values, the wave's counts (wave-uniform: outliers,
// corrections) and the lane's running minima and maxima of the reconstructed
// and the input values (IEEE minimum / maximum: -0 below +0, NaN kept).
struct T0Ctx {
  uint16_t *sc;
  float *exv;          // exact values of the block's level-0 slots, by lane position
  uint32_t nO, nC;
  float rmin, rmax, xmin, xmax;
};

// The quantizer's constants as the tile kernels use them, read once per
// workgroup into scalar registers (readfirstlane: kept in registers rather
// than reloaded from the kernel arguments before every row, where each
// reload's wait would also wait for the row's LDS reads).
struct T0Quant {
  float inv, step, ein, qmaxf;
  double e;
};

__device__ __forceinline__ float sreg(float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); }

__device__ __forceinline__ T0Quant t0_quant(const Geo &gq) {
  T0Quant c;
  c.inv = sreg(gq.inv);
  c.step = sreg(gq.step);
  c.ein = sreg(gq.ein);
  c.qmaxf = sreg((float)gq.qmax);
  const uint64_t eb = __double_as_longlong(gq.e);
  c.e = __longlong_as_double((long long)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)eb)) |
                                         ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(eb >> 32)) << 32)));
  return c;
}

// Ordered key of a binary32 value (as ord_of), in two instructions.
__device__ __forceinline__ uint32_t t0_ord(float f) {
  const uint32_t u = __float_as_uint(f);
  return u ^ ((uint32_t)((int32_t)u >> 31) | 0x80000000u);
}

// OR of v over lanes 0-31 (a) and over lanes 32-63 (b), as wave-uniform
// values: within each 16-lane row (xor 1, xor 2, half mirror, mirror), then
// row 0's result into row 1 and row 2's into row 3 (broadcast of lane 15).
__device__ __forceinline__ void half_or(uint32_t v, uint32_t &a, uint32_t &b) {
  v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xb1, 0xf, 0xf, false);   // quad_perm 1,0,3,2
  v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4e, 0xf, 0xf, false);   // quad_perm 2,3,0,1
  v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xf, 0xf, false);  // row_half_mirror
  v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xf, 0xf, false);  // row_mirror
  v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
  a = (uint32_t)__builtin_amdgcn_readlane((int)v, 31);
  b = (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Quantization, the bound and topology checks, the statistics and the code
// of one point predicted as p, without branches: lanes outside the row hold
// a copy of a point inside it (same value, same code, same LDS slot), so only
// the counts are masked (`cmask`: lanes holding a point of the pair that the
// block owns).  The outlier / correction logic runs on lane masks: a point
// changes side of some candidate exactly when one candidate's comparison
// differs between x and x', so the correction mask is an OR of ballot XORs.
// LL: the lossless quantizer.
// Candidates past K are +inf in `iso` (no finite value reaches them).
template <int KB, bool LL, bool GW = false>
__device__ __forceinline__ void t0_finish(const T0Quant &gq, const float (&iso)[KB], float x, float p, uint64_t cmask,
                                          uint32_t jr, uint32_t jl, T0Ctx &t, char *gl = nullptr,
                                          uint32_t go = 0u) {
  // the point's section index is jr + jl: jr the row's (wave-uniform), jl the lane's
  uint64_t mO;
  float xc;
  int32_t q;
  if (LL) {
    xc = p;
    q = 0;
    mO = __ballot(__float_as_uint(p) != __float_as_uint(x));
  } else {
    const float qf = rintf(__fmul_rn(__fsub_rn(x, p), gq.inv));
    xc = __fadd_rn(p, __fmul_rn(qf, gq.step));
    q = (int32_t)qf;
    const uint64_t mq = __ballot(fabsf(qf) <= gq.qmaxf);
    // the bound in binary32 first; the exact check in double only for a row
    // where some lane is not clearly inside
    uint64_t mb = __ballot(fabsf(__fsub_rn(xc, x)) <= gq.ein);
    if (mb != ~0ull) mb = __ballot(fabs((double)xc - (double)x) <= gq.e);
    mO = ~(mq & mb);
  }
  uint64_t mr = 0;
#pragma unroll
  for (int jj = 0; jj < KB; jj++) mr |= __ballot(iso[jj] <= x) ^ __ballot(iso[jj] <= xc);
  const uint64_t mE = mO | mr;                 // outlier, or a correction (side change, not an outlier)
  const bool E = __builtin_amdgcn_inverse_ballot_w64(mE);
  const float xr = E ? x : xc;
  if (GW) stf(gl, go, xr);                     // above level 0: the parent of the next finer level
  const uint32_t zz = ((uint32_t)q << 1) ^ (uint32_t)(q >> 31);
  t.rmin = __builtin_elementwise_minimum(t.rmin, xr);
  t.rmax = __builtin_elementwise_maximum(t.rmax, xr);
  t.xmin = __builtin_elementwise_minimum(t.xmin, x);
  t.xmax = __builtin_elementwise_maximum(t.xmax, x);
  uint16_t *scr = t.sc + jr;
  scr[jl] = E ? kT0Exact : (uint16_t)zz;
  if (mE) {
    // a row with exact points (rare): the counts, and the exact values into
    // their slots (slot j / 64, lane j % 64)
    t.nO += (uint32_t)__popcll(mO & cmask);
    t.nC += (uint32_t)__popcll(~mO & mr & cmask);
    if (E) t.exv[(size_t)(jr + jl)] = x;
  }
}

// Average along x of parents a0, a1 (xav false: a0 alone), as a select.
__device__ __forceinline__ float t0_xavg(float a0, float a1, bool xav) {
  float m = avg2(a0, a1);
  hold(m);
  return xav ? m : a0;
}

__device__ __forceinline__ float lds_at(const char *base, uint32_t off) {
  return *reinterpret_cast<const float *>(base + off);
}

// Multilinear midpoint of a point of the tile from the staged parent
// planes (rows of Side, planes of Plane floats), any parity (used for the
// few column points).
template <int Side, int Plane>
__device__ __forceinline__ float t0_pred_any(const float *sg, bool zu, uint32_t v, uint32_t u, uint32_t gy,
                                             uint32_t gx) {
  const uint32_t yl = v >> 1, xl = u >> 1;
  const bool yu = (v & 1u) && yl + 1 < gy, xu = (u & 1u) && xl + 1 < gx;
  const uint32_t yb = yu ? yl + 1 : yl, xb = xu ? xl + 1 : xl;
  const float *p1 = zu ? sg + Plane : sg;
  return midpoint8(sg[yl * Side + xl], sg[yl * Side + xb], sg[yb * Side + xl], sg[yb * Side + xb],
                   p1[yl * Side + xl], p1[yl * Side + xb], p1[yb * Side + xl], p1[yb * Side + xb], zu, yu, xu);
}

// Level LV (0 or 1) of 64-cell blocks by pairs of planes of the level's
// grid.  Level 1 is level 0's pattern on every other point of the field,
// x loads at a stride of two, parents from the level-2 grid; its rows hold
// at most 33 points, so a wave instruction takes two rows (lanes 0-31 and
// 32-63, the points u < 32; the points u = 32 go one row per lane, as level
// 0's u = 64) and four of the rows of odd points only.  Its reconstructed
// points, and the level-2 points of the pair's even plane that the level-1
// grid carries over, are written into the level-1 grid for level 0 to
// predict from.
template <int LV>
struct TileDims {
  static constexpr int S = 1 << LV;                       // field points per level step
  static constexpr int Side = (64 >> (LV + 1)) + 1;       // parent points per axis of a block
  static constexpr int Plane = LV == 0 ? 1152 : 320;      // staged parent plane stride (floats)
  static constexpr int Codes = LV == 0 ? 7361 + 63 : 1889 + 63;   // most section points of a pair + a chunk tail
  static constexpr int R = LV == 0 ? 1 : 2;               // full rows per wave instruction
  static constexpr int LW = 64 / R;                       // lanes (points u < LW) of a full row
  static constexpr int QA = 2 * R;                        // rows of odd points (A rows) per wave instruction
  static constexpr int A = LV == 0 ? 5 : 2;               // A-row groups of the even plane per wave
  static constexpr int B = LV == 0 ? 8 : 2;               // odd-row groups of the even plane per wave
  static constexpr int M = LV == 0 ? 9 : 3;               // row-pair groups of the odd plane per wave
};

template <int KB, bool LL, int LV>
__device__ __forceinline__ void encode_tile(const EncPlan &P) {
  using TD = TileDims<LV>;
  constexpr uint32_t S = TD::S;
  constexpr bool GW = LV >= 1;
  // one LDS record with the parent planes first, so that they sit at LDS
  // address 0 and a row's parent offsets fit the read instructions' fields
  struct Lds {
    float sg[2 * TD::Plane];
    uint16_t sc[kT0Spare + TD::Codes + 64];   // + the second chunk of a pair read past the last
    uint32_t pack[kWaves][65];                // + a spare word past the last half
  };
  __shared__ __align__(16) Lds lds;
  float *sg = lds.sg;
  uint16_t *sc = lds.sc;
  uint32_t (*pack)[65] = lds.pack;
  uint32_t w2, b;
  xcd_remap(w2, b);
  const Geo &gq = P.g;
  const BlockPos bp = block_pos(gq, P.l0, b);
  const Sec s = LV == 0 ? P.l0.sec[bp.cls] : P.l0.sec1[bp.cls];
  const SecR rc = LV == 0 ? P.l0.rc[bp.cls] : P.l0.rc1[bp.cls];
  const uint32_t wave = wave_index();
  const int lane = lane_id();
  Part acc;
  part_init(acc);
  Part *rec = &P.part[(int64_t)b * P.part_per_block + (LV == 0 ? 0 : P.part_l1) + w2];
  const uint32_t PP = s.Pe + s.Po;
  const uint32_t J0 = w2 * PP;
  const int64_t slot0 = P.slot_base[LV] + (int64_t)b * P.maxch[LV];
  const uint32_t nch = (s.npts + 63) / 64;
  if (w2 == 0) {
    // slots past this block's section (a shorter block than the first)
    for (uint32_t c = nch + threadIdx.x; c < P.maxch[LV]; c += kBS) P.cnt[slot0 + c] = U4{0, 0, 0, 0};
  }
  if (J0 >= s.npts) {  // a pair past the block's planes
    part_store(acc, rec);
    return;
  }
  const uint32_t we = 2 * w2;                  // the even plane (block-relative, level units)
  const bool has_odd = we + 1 < s.mz;
  const uint32_t J1 = has_odd ? J0 + PP : J0 + s.Pe;
  const uint32_t cfirst = (J0 + 63) / 64, cend = (J1 + 63) / 64;
  const uint32_t jend = min(cend * 64, s.npts);
  const uint32_t jbase = cfirst * 64;          // section index of the tile's first code
  T0Ctx t;
  t.sc = sc + kT0Spare - jbase;                // t.sc[j] for jbase - 63 <= j < jend
  t.exv = P.exv + slot0 * 64;
  t.nO = t.nC = 0;
  t.rmin = t.xmin = __builtin_inff();
  t.rmax = t.xmax = -__builtin_inff();
  const uint32_t n1 = (uint32_t)gq.n[1], n2 = (uint32_t)gq.n[2];
  const uint32_t mx = s.mx, my = s.my, rowE = s.rowE, RP = rowE + mx;
  // the two parent planes (level LV + 1, z = (o_z / S + we) / 2 and the next)
  const uint32_t h0 = (uint32_t)P.gd[LV + 1][0], h1 = (uint32_t)P.gd[LV + 1][1], h2 = (uint32_t)P.gd[LV + 1][2];
  const uint32_t zl0 = (bp.o[0] >> (LV + 1)) + w2, oy1 = bp.o[1] >> (LV + 1), ox1 = bp.o[2] >> (LV + 1);
  const uint32_t gy = (bp.hi[1] >> (LV + 1)) - oy1 + 1, gx = (bp.hi[2] >> (LV + 1)) - ox1 + 1;
  const uint32_t np = zl0 + 1 < h0 ? 2u : 1u;
  // The two parent planes: rows past the block and lanes past a row load
  // (and store) a copy of the last one; without an upper plane the second
  // staged plane is a copy of the first and is never read.  32-bit offsets
  // from the block's first parent.  They are stored into LDS only after the
  // x rows below are loaded, so that both sets of loads are in flight
  // together.
  const uint32_t pxl = min((uint32_t)lane, gx - 1);
  constexpr int kRP = (TD::Side + kWaves - 1) / kWaves;
  float tv[2][kRP];
  {
    const char *__restrict__ g1b =
        reinterpret_cast<const char *>(P.G + P.g_off[LV + 1] + ((size_t)zl0 * h1 + oy1) * h2 + ox1);
    const uint32_t planeB = (np - 1) * h1 * h2 * 4u, rowB1 = h2 * 4u;
#pragma unroll
    for (int pz = 0; pz < 2; pz++)
#pragma unroll
      for (int u = 0; u < kRP; u++) {
        const uint32_t yy = min(wave + (uint32_t)u * kWaves, gy - 1);
        tv[pz][u] = ldf(g1b, (uint32_t)pz * planeB + yy * rowB1 + pxl * 4u);
      }
  }
  float iso[KB];
#pragma unroll
  for (int jj = 0; jj < KB; jj++) iso[jj] = sreg(jj < gq.K ? gq.iso[jj] : __builtin_inff());
  const T0Quant tq = t0_quant(gq);
  // the block's slab of the field; the launcher guarantees it spans < 4 GiB
  const char *__restrict__ xbase = reinterpret_cast<const char *>(P.x + (size_t)bp.o[0] * n1 * n2);
  const char *__restrict__ sgb = reinterpret_cast<const char *>(sg);
  const uint32_t ownz = bp.own[0] - bp.o[0], owny = bp.own[1] - bp.o[1], ownx = bp.own[2] - bp.o[2];
  const bool zu = np == 2;                     // the odd plane has an upper parent plane
  const uint32_t rowB = n2 * 4u * S;           // bytes between the level's rows in the field
  const uint32_t xe0 = ((we * S * n1 + bp.o[1]) * n2 + bp.o[2]) * 4u;  // even plane, row 0
  const uint32_t xo0 = xe0 + n1 * n2 * 4u * S;                      // odd plane, row 0
  // the level's grid (levels >= 1): its rows of the pair's two planes
  const int64_t *gdl = P.gd[LV];
  const uint32_t f1 = GW ? (uint32_t)gdl[1] : 0u, f2 = GW ? (uint32_t)gdl[2] : 0u;
  char *__restrict__ glb =
      GW ? reinterpret_cast<char *>(P.G + P.g_off[LV] +
                                    (((size_t)(bp.o[0] / S) + we) * f1 + bp.o[1] / S) * f2 + bp.o[2] / S)
         : nullptr;
  const uint32_t grow = f2 * 4u, gplane = f1 * f2 * 4u;
  // codes past the section in its last chunk read as 0 when packing
  if (cend > cfirst && cend * 64 > s.npts && threadIdx.x < cend * 64 - s.npts) t.sc[s.npts + threadIdx.x] = 0;
  // and the chunk after the tile's last, which the packing of an odd
  // count of chunks reads as the second of a pair
  if (threadIdx.x < 64) t.sc[cend * 64 + threadIdx.x] = 0;
  // Every x row a wave needs is loaded before the barrier.  Lanes: an A
  // group holds QA rows of odd points (v = 2 (QA a + qa), u = 2 i + 1, lane
  // LA qa + i); a B or C/D group holds R full rows (row R g + hr, u < LW,
  // lane LW hr + uu).  A row past the block or a lane past a row loads (and
  // codes) a copy of a point inside, whose counts are masked.
  constexpr int kA = TD::A, kB = TD::B, kM = TD::M;
  constexpr uint32_t R = TD::R, LW = TD::LW, QA = TD::QA, LA = 64 / QA;
  const uint32_t half = (uint32_t)lane >> 5, ir = (uint32_t)lane & 31u;
  const uint32_t qa = (uint32_t)lane / LA, ia = (uint32_t)lane % LA;
  const uint32_t hr = R == 1 ? 0u : (uint32_t)lane / LW, uu = R == 1 ? (uint32_t)lane : (uint32_t)lane % LW;
  const uint32_t iA = min(ia, rowE > 0 ? rowE - 1 : 0u);
  const uint32_t nEv = (my + 1) / 2;           // even rows of the even plane
  const uint32_t nA = rowE > 0 ? (nEv + QA - 1) / QA : 0u, nB = my / 2, nM = has_odd ? (my + 1) / 2 : 0u;
  const uint32_t u = min(uu, mx - 1);
  const uint32_t lxA = (2 * iA + 1) * 4u * S, lx = u * 4u * S;
  // the row of A group a for this lane (a sub-row past the plane: the group's first)
  auto a_row = [&](uint32_t a) {
    const uint32_t v = 2 * (QA * a + qa);
    return v < my ? v : 2 * QA * a;
  };
  // lanes of sub-row h of a group of n sub-rows (wave-uniform masks)
  auto sub_lanes = [](uint32_t h, uint32_t n) -> uint64_t {
    return n == 1 ? ~0ull : (((1ull << (64 / n)) - 1ull) << (h * (64 / n)));
  };
  float xa[kA], xb[kB], xc[kM], xd[kM];
  if (nA > 0) {
#pragma unroll
    for (int k = 0; k < kA; k++) {
      const uint32_t a = min(wave + (uint32_t)k * kWaves, nA - 1);
      xa[k] = ldf(xbase, xe0 + a_row(a) * rowB + lxA);
    }
  }
  if (nB > 0) {
#pragma unroll
    for (int k = 0; k < kB; k++) {
      const uint32_t f = min(R * (wave + (uint32_t)k * kWaves) + hr, nB - 1);
      xb[k] = ldf(xbase, xe0 + (2 * f + 1) * rowB + lx);
    }
  }
  if (nM > 0) {
#pragma unroll
    for (int k = 0; k < kM; k++) {
      const uint32_t m = min(R * (wave + (uint32_t)k * kWaves) + hr, nM - 1);
      xc[k] = ldf(xbase, xo0 + 2 * m * rowB + lx);
      xd[k] = ldf(xbase, xo0 + min(2 * m + 1, my - 1) * rowB + lx);
    }
  }
#pragma unroll
  for (int pz = 0; pz < 2; pz++)
#pragma unroll
    for (int u = 0; u < kRP; u++) {
      const uint32_t yy = min(wave + (uint32_t)u * kWaves, gy - 1);
      sg[pz * TD::Plane + yy * TD::Side + pxl] = tv[pz][u];
    }
  __syncthreads();

  if (GW) {
    // the parents on the even plane's even rows and even points carry over
    // into the level's grid unchanged
    for (uint32_t r = wave; 2 * r < my; r += kWaves)
      if (ir < gx && half == 0) stf(glb, 2 * r * grow + 2 * ir * 4u, sg[r * TD::Side + ir]);
  }
  // ---- A rows: even plane, even rows v, odd u = 2i + 1
  if (nA > 0) {
    const bool xav = iA + 1 < gx;
    const uint64_t lane_inA = __ballot(ia < rowE && (2 * ia + 1) * S < ownx);
    const uint32_t lg = iA * 4u;
#pragma unroll
    for (int k = 0; k < kA; k++) {
      const uint32_t a = wave + (uint32_t)k * kWaves;
      if (a >= nA) break;
      const uint32_t vc = a_row(a);
      const uint32_t ga = (vc >> 1) * (TD::Side * 4u) + lg;
      const float p = t0_xavg(lds_at(sgb, ga), lds_at(sgb, ga + 4), xav);
      const uint32_t jA = J0 + (vc >> 1) * RP;
      uint64_t rows = 0;
#pragma unroll
      for (uint32_t h = 0; h < QA; h++) {
        const uint32_t vh = 2 * (QA * a + h);
        if (vh < my && vh * S < owny) rows |= sub_lanes(h, QA);
      }
      const uint64_t cm = we * S < ownz ? lane_inA & rows : 0ull;
      t0_finish<KB, LL, GW>(tq, iso, xa[k], p, cm, jA, iA, t, glb, vc * grow + (2 * iA + 1) * 4u);
    }
  }
  const uint32_t lx0 = u >> 1;
  const bool xav = (u & 1u) && lx0 + 1 < gx;
  const uint64_t lane_in = __ballot(uu < mx && uu * S < ownx);
  const uint32_t lg = lx0 * 4u;
  constexpr uint32_t kRow = TD::Side * 4u, kPl = TD::Plane * 4u;
  // ---- B rows: odd rows v = 2f + 1 of the even plane (z even, y odd)
#pragma unroll
  for (int k = 0; k < kB; k++) {
    const uint32_t f0 = R * (wave + (uint32_t)k * kWaves);
    if (f0 >= nB) break;
    const uint32_t f = R == 1 ? f0 : min(f0 + hr, nB - 1);
    const bool yu = f + 1 < gy;
    const uint32_t ga = f * kRow + lg;
    // the row's parents read together, before any value is used
    const float a0 = lds_at(sgb, ga), a1 = lds_at(sgb, ga + 4);
    const float b0 = lds_at(sgb, ga + kRow), b1 = lds_at(sgb, ga + kRow + 4);
    const float A = t0_xavg(a0, a1, xav);
    const float B = t0_xavg(b0, b1, xav);
    float pb = avg2(A, B);
    hold(pb);
    const float p = yu ? pb : A;
    const uint32_t jr = J0 + f * RP + rowE;
    uint64_t rows = 0;
#pragma unroll
    for (uint32_t h = 0; h < R; h++)
      if (f0 + h < nB && (2 * (f0 + h) + 1) * S < owny) rows |= sub_lanes(h, R);
    const uint64_t cm = we * S < ownz ? lane_in & rows : 0ull;
    t0_finish<KB, LL, GW>(tq, iso, xb[k], p, cm, jr, u, t, glb, (2 * f + 1) * grow + u * 4u);
  }
  // ---- C and D rows: the odd plane's rows 2m (y even) and 2m + 1 (y odd)
  {
    const uint32_t jo = J0 + s.Pe;
    const bool zown = (we + 1) * S < ownz;
#pragma unroll
    for (int k = 0; k < kM; k++) {
      const uint32_t m0 = R * (wave + (uint32_t)k * kWaves);
      if (m0 >= nM) break;
      const uint32_t m = R == 1 ? m0 : min(m0 + hr, nM - 1);
      uint64_t rowsC = 0, rowsD = 0;
#pragma unroll
      for (uint32_t h = 0; h < R; h++) {
        const uint32_t mh = m0 + h;
        if (mh < nM && 2 * mh * S < owny) rowsC |= sub_lanes(h, R);
        if (mh < nM && 2 * mh + 1 < my && (2 * mh + 1) * S < owny) rowsD |= sub_lanes(h, R);
      }
      const uint32_t ga = m * kRow + lg;
      // the parents of both rows read together, before any value is used
      // (rows m + 1 past the plane read the staging's spare floats, unused)
      const float a0 = lds_at(sgb, ga), a1 = lds_at(sgb, ga + 4);
      const float c0 = lds_at(sgb, ga + kPl), c1 = lds_at(sgb, ga + kPl + 4);
      const float b0 = lds_at(sgb, ga + kRow), b1 = lds_at(sgb, ga + kRow + 4);
      const float d0 = lds_at(sgb, ga + kPl + kRow), d1 = lds_at(sgb, ga + kPl + kRow + 4);
      const float A = t0_xavg(a0, a1, xav);
      const float Cc = t0_xavg(c0, c1, xav);
      float pc = avg2(A, Cc);
      hold(pc);
      const float p = zu ? pc : A;
      const uint32_t jc = jo + 2 * m * mx;
      t0_finish<KB, LL, GW>(tq, iso, xc[k], p, zown ? lane_in & rowsC : 0ull, jc, u, t, glb,
                            gplane + 2 * m * grow + u * 4u);
      if (R == 1 ? 2 * m + 1 < my : 2 * m0 + 1 < my) {
        const bool yu = m + 1 < gy;
        const float B = t0_xavg(b0, b1, xav);
        const float D = t0_xavg(d0, d1, xav);
        float p0 = avg2(A, B), p1 = avg2(Cc, D);
        hold(p0);
        hold(p1);
        p0 = yu ? p0 : A;
        p1 = yu ? p1 : Cc;
        float pd = avg2(p0, p1);
        hold(pd);
        float p2 = zu ? pd : p0;
        uint32_t jd = jc + mx, gd = gplane + (2 * m + 1) * grow + u * 4u;
        if (R > 1) {
          // a lane whose row 2m + 1 is past the plane codes its row 2m again
          // (its x loads are row 2m's): same code into the same slot, not
          // counted
          const bool dok = 2 * m + 1 < my;
          p2 = dok ? p2 : p;
          jd = dok ? jd : jc;
          gd = dok ? gd : gplane + 2 * m * grow + u * 4u;
        }
        t0_finish<KB, LL, GW>(tq, iso, xd[k], p2, zown ? lane_in & rowsD : 0ull, jd, u, t, glb, gd);
      }
    }
  }
  // ---- column: the points u = LW of the full rows (rows of LW + 1 points)
  const uint32_t nF = nB + (has_odd ? my : 0u);
  if (mx == LW + 1) {
    for (uint32_t c0 = wave * 64; c0 < nF; c0 += kWaves * 64) {
      const uint32_t fr = c0 + (uint32_t)lane, f = min(fr, nF - 1);
      const bool ev = f < nB;
      const uint32_t w = ev ? we : we + 1, v = ev ? 2 * f + 1 : f - nB;
      const float x = ldf(xbase, ((w * S * n1 + bp.o[1] + v * S) * n2 + bp.o[2] + LW * S) * 4u);
      const float p = t0_pred_any<TD::Side, TD::Plane>(sg, (w & 1u) && zu, v, LW, gy, gx);
      const uint32_t j = ev ? J0 + (v >> 1) * RP + rowE + LW : J0 + s.Pe + v * mx + LW;
      t0_finish<KB, LL, GW>(tq, iso, x, p, __ballot(fr < nF && w * S < ownz && v * S < owny && LW * S < ownx), 0u, j,
                            t, glb, (ev ? 0u : gplane) + v * grow + LW * 4u);
    }
  }
  // ---- the tail of the last chunk (the next planes' first points; more
  // than one pair when a pair holds fewer than 64 points), parents read from
  // the parent grid in memory; not counted and not written to the level's
  // grid (the next pairs count and write them)
  if (jend > J1 && jbase < jend && wave == kWaves - 1) {
    const uint32_t j = min(J1 + (uint32_t)lane, jend - 1);
    uint32_t w, v, uu2;
    sec_point24(s, rc, j, w, v, uu2);
    const float x = ldf(xbase, ((w * S * n1 + bp.o[1] + v * S) * n2 + bp.o[2] + uu2 * S) * 4u);
    const float p = predict(P.G + P.g_off[LV + 1], h0, h1, h2, LV, bp.o[0] + w * S, bp.o[1] + v * S,
                            bp.o[2] + uu2 * S);
    t0_finish<KB, LL>(tq, iso, x, p, 0ull, 0u, j, t);
  }
  __syncthreads();

  // ---- pack the pair's chunks from LDS into their slots (exact values are
  // already in the slots, at their lanes: count word 3 says so), two chunks
  // at a time: lane i reads the codes 2i and 2i + 1 of chunks c, c + 1 (c
  // even from cfirst) as one word, so lanes 0-31 hold chunk c and lanes
  // 32-63 chunk c + 1; one OR reduction gives both widths, and each chunk
  // packs into its own half of the wave's LDS row (at most 2 * 16 words:
  // codes are below 2^16 - 1).  The wave takes the chunk pairs
  // cfirst + 2 (wave + 4k); the counts of its pair k wait in lane k of a
  // register (chunk c in the low half-word, c + 1 in the high one) and are
  // stored together after the loop.
  uint32_t *pk = pack[wave];                   // 64 words, every lane clears its own
  char *__restrict__ payw = reinterpret_cast<char *>(P.pay + slot0 * 32);
  const uint32_t nchk = cend > cfirst ? cend - cfirst : 0u;
  const uint32_t npair = (nchk + 1) / 2;
  const uint32_t nmine = npair > wave ? (npair - wave + kWaves - 1) / kWaves : 0u;
  const uint32_t lh = (uint32_t)lane & 31u;    // the lane's place in its chunk's half
  uint32_t *pkh = pk + (half << 5);
  uint32_t cw = 0;                             // lane k: width | exact points << 5, per chunk of pair k
  for (uint32_t k = 0; k < nmine; k++) {
    const uint32_t c = cfirst + 2 * (wave + k * kWaves);
    // chunk c + 1 past the tile's last reads zeros
    const uint32_t v2 = *reinterpret_cast<const uint32_t *>(t.sc + c * 64 + 2 * (uint32_t)lane);
    uint32_t lo = v2 & 0xffffu, hi = v2 >> 16;
    uint32_t wA = 0u, wB = 0u;
    uint64_t emA = 0ull, emB = 0ull;
    if (__ballot(v2 != 0u)) {
      // the chunks' widths: bit lengths of the OR of each half's codes (a
      // chunk of zero codes, common, has width 0 and no payload); an exact
      // point's marker sets bit 15, so only then are the exact points
      // looked for (their masks in code order) and taken out of the widths
      uint32_t oA, oB;
      half_or(lo | hi, oA, oB);
      if ((oA | oB) & 0x8000u) {
        emA = __ballot(t.sc[c * 64 + (uint32_t)lane] == kT0Exact);
        emB = __ballot(t.sc[c * 64 + 64 + (uint32_t)lane] == kT0Exact);
        lo = lo == kT0Exact ? 0u : lo;
        hi = hi == kT0Exact ? 0u : hi;
        half_or(lo | hi, oA, oB);
      }
      wA = oA ? 32u - (uint32_t)__clz((int)oA) : 0u;
      wB = oB ? 32u - (uint32_t)__clz((int)oB) : 0u;
      const uint32_t wl = half ? wB : wA;
      pk[lane] = 0u;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      // the lane's two codes (2 wl bits) at bit 2 lh wl of its half: the
      // word holding the start, and the next one (its top `bit mod 32`
      // bits, an extract of width 0 when the start is word-aligned; the
      // word past a half is the next half's first or the row's spare, and
      // only zeros reach it)
      const uint32_t pv = lo | (hi << wl);
      const uint32_t bit = mul24v(2 * lh, wl);
      uint32_t *dst = pkh + (bit >> 5);
      __hip_atomic_fetch_or(dst, pv << (bit & 31u), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
      __hip_atomic_fetch_or(dst + 1, __builtin_amdgcn_ubfe(pv, 0u - bit, bit), __ATOMIC_RELAXED,
                            __HIP_MEMORY_SCOPE_WAVEFRONT);
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
      if ((lh >> 1) < wl) stu(payw, (c * 32 + (uint32_t)lane) * 4u, pk[lane]);
    }
    wA = (uint32_t)__builtin_amdgcn_readfirstlane(wA);
    wB = (uint32_t)__builtin_amdgcn_readfirstlane(wB);
    writelane(cw, wA | ((uint32_t)__popcll(emA) << 5) | ((wB | ((uint32_t)__popcll(emB) << 5)) << 16), k);
    if (emA && lane == 0) P.emask[slot0 + c] = emA;
    if (emB && lane == 0) P.emask[slot0 + c + 1] = emB;
    __builtin_amdgcn_wave_barrier();
  }
  {
    const uint32_t i = (uint32_t)lane, c = cfirst + 2 * (wave + (i >> 1) * kWaves) + (i & 1u);
    const uint32_t w = (uint32_t)__shfl((int)cw, (int)(i >> 1), kWave) >> (16 * (i & 1u));
    if (i < 2 * nmine && c < cend) {
      const uint32_t ne = (w >> 5) & 0x7fu, he = ne ? 1u : 0u;
      P.cnt[slot0 + c] = U4{w & 31u, he, ne, he};
    }
  }
  // the lane's extremes as order-preserving keys (a lane that saw no point
  // keeps +inf / -inf, which no finite value loses to); a non-finite input
  // shows as an infinite extreme or a NaN; the wave's counts join the lane
  // records once per wave
  acc.rmin = t0_ord(t.rmin); acc.rmax = t0_ord(t.rmax);
  acc.xmin = t0_ord(t.xmin); acc.xmax = t0_ord(t.xmax);
  acc.nonfinite = (t.xmin > -__builtin_inff() && t.xmax < __builtin_inff()) ? 0u : 1u;
  if (lane == 0) {
    acc.nO = t.nO;
    acc.nC = t.nC;
  }
  part_store(acc, rec);
}

template <int KB, bool LL>
__global__ __launch_bounds__(kBS) void k_encode_l0t(EncPlan P) {
  encode_tile<KB, LL, 0>(P);
}

template <int KB, bool LL>
__global__ __launch_bounds__(kBS) void k_encode_l1t(EncPlan P) {
  encode_tile<KB, LL, 1>(P);
}

// ------------------------------------------------ levels L .. 2 in one pass
//
// The levels of a 64-cell block from the anchors down to level 2 hold at
// most 17^3 points (the block's points of the 4-grid).  One workgroup per
// block: each thread owns fixed 4-grid points (coordinates by constant
// divisions, a point's level from its coordinates' trailing zeros), reads
// their input once and keeps it in registers.  Level by level, coarsest
// first, a thread's points of that level predict from the reconstructed
// coarser points in LDS, quantize and check as everywhere else, leave their
// reconstruction in LDS and their code at their section index (in closed
// form from the coordinates) in an LDS code array.  Then the chunks of every
// level are packed into their slots and the reconstructed 4-grid is written
// to the level-2 grid, where level 1 predicts from it.

template <int KB>
__global__ __launch_bounds__(kTopBS) void k_encode_top(EncPlan P) {
  __shared__ float R[kTopPts];                 // the reconstruction at the block's 4-grid points
  __shared__ uint16_t sc[kTopCodes];
  __shared__ uint32_t pack[kTopWaves][64];
  __shared__ Part red[kTopWaves];
  __shared__ uint32_t base[kMaxLevels], npt[kMaxLevels];   // each level's first code and points
  const uint32_t b = blockIdx.x;
  const Geo &gq = P.g;
  const int L = gq.nL - 1;
  const BlockPos bp = block_pos(gq, P.l0, b);
  const uint32_t wave = wave_index();
  const int lane = lane_id();
  const uint32_t n1 = (uint32_t)gq.n[1], n2 = (uint32_t)gq.n[2];
  const uint32_t d0 = ((bp.hi[0] - bp.o[0]) >> 2) + 1, d1 = ((bp.hi[1] - bp.o[1]) >> 2) + 1;
  const uint32_t d2 = ((bp.hi[2] - bp.o[2]) >> 2) + 1;
  // the thread's points: coordinates and level packed in one word (x, y, z
  // in bits 0-4, 5-9, 10-14, level + 1 from bit 15, 0 for no point), input
  // (all loads in flight)
  uint32_t pc[kTopPer];
  float xv[kTopPer];
  {
    const char *__restrict__ xbase = reinterpret_cast<const char *>(P.x + (size_t)bp.o[0] * n1 * n2);
#pragma unroll
    for (int k = 0; k < kTopPer; k++) {
      pc[k] = top_point(threadIdx.x + (uint32_t)k * kTopBS, d0, d1, d2, L);
      const uint32_t xc = pc[k] & 31u, yc = (pc[k] >> 5) & 31u, zc = (pc[k] >> 10) & 31u;
      xv[k] = ldf(xbase, ((4 * zc * n1 + bp.o[1] + 4 * yc) * n2 + bp.o[2] + 4 * xc) * 4u);
    }
  }
  if (threadIdx.x == 0) {
    uint32_t off = 0;
    for (int l = L; l >= 2; l--) {
      const uint32_t n = sec_dims(bp, l, L).npts;
      base[l] = off;
      npt[l] = n;
      off += (n + 63) & ~63u;
    }
  }
  float iso[KB];
#pragma unroll
  for (int jj = 0; jj < KB; jj++) iso[jj] = gq.iso[jj];
  Part acc;
  part_init(acc);
  uint32_t nO = 0, nC = 0;
  __syncthreads();
  // ---- the levels, coarsest first
  for (int l = L; l >= 2; l--) {
    const SecDims sd = sec_dims(bp, l, L);
    const uint32_t sh = (uint32_t)(l - 2), st = 1u << sh;     // the level's step on the 4-grid
    const int64_t slot0 = P.slot_base[l] + (int64_t)b * P.maxch[l];
    const uint32_t bl = base[l];
#pragma unroll
    for (int k = 0; k < kTopPer; k++) {
      if ((pc[k] >> 15) != (uint32_t)(l + 1)) continue;
      const uint32_t x = pc[k] & 31u, y = (pc[k] >> 5) & 31u, z = (pc[k] >> 10) & 31u;
      const uint32_t w = z >> sh, v = y >> sh, u = x >> sh;
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
      int32_t q;
      int O, C = 0;
      float xr;
      quantize(gq, xv[k], p, q, O, xr);
      if (!O && gq.K > 0) C = rank_of<KB>(iso, gq.K, xv[k]) != rank_of<KB>(iso, gq.K, xr);
      const bool E = O || C;
      if (E) { xr = xv[k]; q = 0; }
      R[top_idx(z, y, x)] = xr;
      const uint32_t j = sec_index(sd, l == L, w, v, u);
      sc[bl + j] = E ? kT0Exact : (uint16_t)(((uint32_t)q << 1) ^ (uint32_t)(q >> 31));
      if (E) P.exv[slot0 * 64 + j] = xv[k];   // slot j / 64, lane j % 64
      const uint32_t ro = ord_of(xr), xo = ord_of(xv[k]);
      acc.rmin = min(acc.rmin, ro); acc.rmax = max(acc.rmax, ro);
      acc.xmin = min(acc.xmin, xo); acc.xmax = max(acc.xmax, xo);
      acc.nonfinite |= !isfinite(xv[k]);
      if (bp.o[0] + 4 * z < bp.own[0] && bp.o[1] + 4 * y < bp.own[1] && bp.o[2] + 4 * x < bp.own[2]) {
        nO += (uint32_t)O;
        nC += (uint32_t)C;
      }
    }
    // codes past the section in its last chunk read as 0 when packing
    const uint32_t pad = ((sd.npts + 63) & ~63u) - sd.npts;
    if (threadIdx.x < pad) sc[bl + sd.npts + threadIdx.x] = 0;
    __syncthreads();
  }
  // ---- pack every level's chunks into their slots (exact values are already
  // in the slots, at their lanes: count word 3 says so); slots past a
  // section (a shorter block than the first) get zero counts
  uint32_t *pk = pack[wave];
  for (int l = L; l >= 2; l--) {
    const uint32_t nch = (npt[l] + 63) / 64, bl = base[l];
    const int64_t slot0 = P.slot_base[l] + (int64_t)b * P.maxch[l];
    for (uint32_t c = nch + threadIdx.x; c < P.maxch[l]; c += kTopBS) P.cnt[slot0 + c] = U4{0, 0, 0, 0};
    char *__restrict__ payw = reinterpret_cast<char *>(P.pay + slot0 * 32);
    for (uint32_t c = wave; c < nch; c += kTopWaves) {
      const uint32_t v16 = sc[bl + c * 64 + (uint32_t)lane];
      const uint64_t em = __ballot(v16 == kT0Exact);
      const uint32_t zz = __builtin_amdgcn_inverse_ballot_w64(em) ? 0u : v16;
      const uint32_t orv = wave_or_dpp(zz);
      const uint32_t wb = orv ? 32u - (uint32_t)__clz((int)orv) : 0u;
      pk[lane] = 0u;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      if (zz) {
        const uint32_t bit = mul24s((uint32_t)lane, wb), wi = bit >> 5, off = bit & 31u;
        __hip_atomic_fetch_or(&pk[wi], zz << off, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        if (off + wb > 32u)
          __hip_atomic_fetch_or(&pk[wi + 1], zz >> (32u - off), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
      if ((uint32_t)lane < 2 * wb) stu(payw, (c * 32 + (uint32_t)lane) * 4u, pk[lane]);
      if (lane == 0) {
        const uint32_t he = em ? 1u : 0u;
        P.cnt[slot0 + c] = U4{wb, he, (uint32_t)__popcll(em), he};
        if (em) P.emask[slot0 + c] = em;
      }
      __builtin_amdgcn_wave_barrier();
    }
  }
  // ---- the reconstructed 4-grid into the level-2 grid (every point of the
  // closed extent; neighbours write their shared faces with the same values)
  {
    const int64_t *g2 = P.gd[2];
    const uint32_t e1 = (uint32_t)g2[1], e2 = (uint32_t)g2[2];
    char *__restrict__ gb =
        reinterpret_cast<char *>(P.G + P.g_off[2] + (((size_t)(bp.o[0] >> 2)) * e1 + (bp.o[1] >> 2)) * e2 + (bp.o[2] >> 2));
#pragma unroll
    for (int k = 0; k < kTopPer; k++)
      if (pc[k] >> 15) {
        const uint32_t x = pc[k] & 31u, y = (pc[k] >> 5) & 31u, z = (pc[k] >> 10) & 31u;
        stf(gb, ((z * e1 + y) * e2 + x) * 4u, R[top_idx(z, y, x)]);
      }
  }
  // the block's record: lanes, then waves, then one thread
  Part r;
  r.rmin = wave_min_dpp(acc.rmin); r.rmax = wave_max_dpp(acc.rmax);
  r.xmin = wave_min_dpp(acc.xmin); r.xmax = wave_max_dpp(acc.xmax);
  r.nonfinite = wave_or_dpp(acc.nonfinite); r.nO = wave_sum_dpp(nO); r.nC = wave_sum_dpp(nC);
  r.pad = 0;
  if (lane == 0) red[wave] = r;
  __syncthreads();
  if (threadIdx.x == 0) {
    Part t = red[0];
    for (int i = 1; i < kTopWaves; i++) {
      t.rmin = min(t.rmin, red[i].rmin); t.rmax = max(t.rmax, red[i].rmax);
      t.xmin = min(t.xmin, red[i].xmin); t.xmax = max(t.xmax, red[i].xmax);
      t.nonfinite |= red[i].nonfinite; t.nO += red[i].nO; t.nC += red[i].nC;
    }
    P.part[(int64_t)b * P.part_per_block + (P.part_per_block - 1)] = t;
  }
}

// Differentiated error control: block b is active when the input on its
// closed extent crosses a candidate isovalue (min < k <= max).  Workgroup
// (s, b) reduces planes s, s + kActSplit, ... of block b's extent (each
// thread four points at a time, loads issued together) into partial
// order-preserving min/max keys; k_block_active_final combines them.

__global__ __launch_bounds__(kBS) void k_block_minmax(EncPlan P) {
  __shared__ uint32_t red[kWaves][2];
  const Geo &g = P.g;
  const int64_t b = blockIdx.y;
  int64_t o[3], hi[3];
  block_ext(g, b, o, hi);
  const uint32_t nz = (uint32_t)(hi[0] - o[0] + 1), ny = (uint32_t)(hi[1] - o[1] + 1), nx = (uint32_t)(hi[2] - o[2] + 1);
  const uint32_t plane = ny * nx;
  const size_t n1 = (size_t)g.n[1], n2 = (size_t)g.n[2];
  uint32_t mn = 0xffffffffu, mx = 0u;
  for (uint32_t z = blockIdx.x; z < nz; z += kActSplit) {
    const float *pz = P.x + ((size_t)(o[0] + z) * n1 + (size_t)o[1]) * n2 + (size_t)o[2];
    for (uint32_t i0 = threadIdx.x; i0 < plane; i0 += 4 * kBS) {
      float v[4];
#pragma unroll
      for (int u = 0; u < 4; u++) {
        const uint32_t i = min(i0 + (uint32_t)u * kBS, plane - 1);  // repeats a point: harmless for min/max
        const uint32_t y = i / nx, x = i - y * nx;
        v[u] = pz[(size_t)y * n2 + x];
      }
#pragma unroll
      for (int u = 0; u < 4; u++) {
        const uint32_t k = ord_of(v[u]);
        mn = min(mn, k);
        mx = max(mx, k);
      }
    }
  }
  mn = wave_min_u(mn);
  mx = wave_max_u(mx);
  const int wave = threadIdx.x / kWave;
  if (lane_id() == 0) { red[wave][0] = mn; red[wave][1] = mx; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < kWaves; i++) { mn = min(mn, red[i][0]); mx = max(mx, red[i][1]); }
    uint32_t *part = P.act + g.nblocks + 2 * (b * kActSplit + blockIdx.x);
    part[0] = mn;
    part[1] = mx;
  }
}

__global__ __launch_bounds__(kBS) void k_block_active_final(EncPlan P) {
  const Geo &g = P.g;
  const int64_t b = (int64_t)blockIdx.x * kBS + threadIdx.x;
  if (b >= g.nblocks) return;
  uint32_t mn = 0xffffffffu, mx = 0u;
  for (int s2 = 0; s2 < kActSplit; s2++) {
    const uint32_t *part = P.act + g.nblocks + 2 * (b * kActSplit + s2);
    mn = min(mn, part[0]);
    mx = max(mx, part[1]);
  }
  const float vmn = of_ord(mn), vmx = of_ord(mx);
  uint32_t a = 0;
  for (int j = 0; j < g.K; j++) a |= (vmn < g.iso[j] && g.iso[j] <= vmx) ? 1u : 0u;
  P.act[b] = a;
}

// Block merging before compression: the index signature of every block, bit
// j set when the input on its closed extent crosses candidate j
// (min < k_j <= max), from k_block_minmax's partial keys.
__global__ __launch_bounds__(kBS) void k_block_sig(EncPlan P) {
  const Geo &g = P.g;
  const int64_t b = (int64_t)blockIdx.x * kBS + threadIdx.x;
  if (b >= g.nblocks) return;
  uint32_t mn = 0xffffffffu, mx = 0u;
  for (int s2 = 0; s2 < kActSplit; s2++) {
    const uint32_t *part = P.act + g.nblocks + 2 * (b * kActSplit + s2);
    mn = min(mn, part[0]);
    mx = max(mx, part[1]);
  }
  const float vmn = of_ord(mn), vmx = of_ord(mx);
  uint32_t sig = 0;
  for (int j = 0; j < g.K; j++) sig |= (vmn < g.iso[j] && g.iso[j] <= vmx) ? 1u << j : 0u;
  P.act[b] = sig;
}

// Byte size of every section from the scanned chunk sizes.
__global__ __launch_bounds__(kBS) void k_sections(EncPlan P) {
  const Geo &g = P.g;
  const int64_t nsec = g.nblocks * g.nL;
  const int64_t sec = (int64_t)blockIdx.x * kBS + threadIdx.x;
  if (sec >= nsec) return;
  const int L = g.nL - 1;
  const int64_t b = sec / g.nL;
  const int l = L - (int)(sec % g.nL);
  int64_t o[3], hi[3];
  unit_ext(g, b, o, hi);
  const Sec s = sec_geom(o, hi, l, L);
  const uint32_t nch = (s.npts + 63) / 64;
  const int64_t s0 = slot_of(P, l, b);
  const U4 a = P.P[s0], e = P.P[s0 + nch];
  P.secsz[sec] = sec_bytes(s.npts, e.x - a.x, e.y - a.y, e.z - a.z);
}

__device__ inline void put8(const EncPlan &P, uint64_t off, uint8_t v) {
  if (off < P.cap) P.out[off] = v;
}
__device__ inline void put32(const EncPlan &P, uint64_t off, uint32_t v) {
  if (off + 4 <= P.cap) *reinterpret_cast<uint32_t *>(P.out + off) = v;
}
__device__ inline void put64(const EncPlan &P, uint64_t off, uint64_t v) {
  if (off + 8 <= P.cap) {
    uint32_t *p = reinterpret_cast<uint32_t *>(P.out + off);
    p[0] = (uint32_t)v;
    p[1] = (uint32_t)(v >> 32);
  }
}

// Box table of a merged stream: the unit table, after the block table.
__global__ __launch_bounds__(kBS) void k_box_table(EncPlan P) {
  const Geo &g = P.g;
  const int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x;
  if (i >= 8 * g.nblocks) return;
  put32(P, P.payload_off - 32 * (uint64_t)g.nblocks + 4 * (uint64_t)i, g.units[i]);
}

// Section table entries, section headers and padding bytes.
__global__ __launch_bounds__(kBS) void k_sec_table(EncPlan P) {
  const Geo &g = P.g;
  const int64_t nsec = g.nblocks * g.nL;
  const int64_t sec = (int64_t)blockIdx.x * kBS + threadIdx.x;
  if (sec >= nsec) return;
  const int L = g.nL - 1;
  const int64_t b = sec / g.nL;
  const int l = L - (int)(sec % g.nL);
  int64_t o[3], hi[3];
  unit_ext(g, b, o, hi);
  const Sec s = sec_geom(o, hi, l, L);
  const uint32_t nch = (s.npts + 63) / 64, ntile = (nch + 63) / 64;
  const int64_t s0 = slot_of(P, l, b);
  const U4 a = P.P[s0], e = P.P[s0 + nch];
  const uint32_t W = e.x - a.x, NE = e.y - a.y, NX = e.z - a.z;
  const uint64_t so = P.payload_off + P.secoff[sec];
  put64(P, kHeaderBytes + 16 * (uint64_t)sec, so);
  put64(P, kHeaderBytes + 16 * (uint64_t)sec + 8, P.secsz[sec]);
  put32(P, so, s.npts);
  put32(P, so + 4, W);
  put32(P, so + 8, NE);
  put32(P, so + 12, NX);
  const uint64_t tt = 16 + 12 * (uint64_t)ntile, A = 16 + pad8(12 * (uint64_t)ntile);
  for (uint64_t i = tt; i < A; i++) put8(P, so + i, 0);
  const uint64_t H = A + nch, Poff = A + pad8(nch);
  for (uint64_t i = H; i < Poff; i++) put8(P, so + i, 0);
  const uint64_t Xend = Poff + 8 * (uint64_t)W + 8 * (uint64_t)NE + 4 * (uint64_t)NX;
  const uint64_t end = Poff + 8 * (uint64_t)W + 8 * (uint64_t)NE + pad8(4 * (uint64_t)NX);
  for (uint64_t i = Xend; i < end; i++) put8(P, so + i, 0);
}

// Copies the chunks of one tile (64 chunks) of one section from their slots
// into the stream: chunk header bytes, the tile-table entry, payload words,
// exact masks and exact values.  Payload words are flattened over the tile,
// so consecutive threads move consecutive 8-byte words of the stream.  One
// workgroup per (level, block, tile); levels are laid out from the coarsest
// (first workgroups) to level 0.  A section that does not fit the capacity is
// not written (the result then reports the required size).
constexpr int kPackUnroll = 8;

__global__ __launch_bounds__(kBS) void k_pack(EncPlan P) {
  // source of each payload word of the tile: its chunk (within the tile)
  // times 16 plus its place in the chunk's slot
  __shared__ uint16_t s_src_all[kWaves][64 * kMaxW];
  const Geo &g = P.g;
  const int L = g.nL - 1;
  const int lane = lane_id();
  const uint32_t wave = wave_index();
  uint16_t *s_src = s_src_all[wave];
  // one wave per tile of 64 chunks (tiles of every section in level-major order)
  const int64_t wg = (int64_t)blockIdx.x * kWaves + wave;
  if (wg >= P.pack_base[0] + g.nblocks * P.pack_gpb[0]) return;
  int l = L;
  for (int t = L - 1; t >= 0; t--)
    if (wg >= P.pack_base[t]) l = t;
  const int64_t rel = wg - P.pack_base[l];
  const int64_t b = rel / P.pack_gpb[l];
  const uint32_t tile = (uint32_t)(rel - b * P.pack_gpb[l]);
  Sec s;
  if (l == 0 && !g.units) {
    s = P.l0.sec[block_pos(g, P.l0, (uint32_t)b).cls];
  } else if (l == 1 && !g.units) {
    s = P.l0.sec1[block_pos(g, P.l0, (uint32_t)b).cls];
  } else {
    int64_t o[3], hi[3];
    unit_ext(g, b, o, hi);
    s = sec_geom(o, hi, l, L);
  }
  const uint32_t nch = (s.npts + 63) / 64;
  const uint32_t ntile = (nch + 63) / 64;
  if (tile >= ntile) return;
  const int64_t sec = b * g.nL + (L - l);
  const uint64_t so = P.payload_off + P.secoff[sec];
  if (so + P.secsz[sec] > P.cap) return;
  const int64_t s0 = slot_of(P, l, b);
  const U4 a = P.P[s0], e = P.P[s0 + nch];
  const uint32_t W = e.x - a.x, NE = e.y - a.y;
  const uint64_t A = 16 + pad8(12 * (uint64_t)ntile), Poff = A + pad8(nch);
  const uint64_t Moff = Poff + 8 * (uint64_t)W, Xoff = Moff + 8 * (uint64_t)NE;
  const uint32_t c0 = tile * 64, tn = min(64u, nch - c0);
  uint8_t *out = P.out + so;
  const int64_t slot0 = s0 + c0;
  const bool on = (uint32_t)lane < tn;
  const U4 cur = on ? P.P[slot0 + lane] : U4{0, 0, 0, 0};
  const U4 cc = on ? P.cnt[slot0 + lane] : U4{0, 0, 0, 0};
  const unsigned long long em = (on && cc.y) ? P.emask[slot0 + lane] : 0ull;
  const uint32_t base_w = __builtin_amdgcn_readfirstlane(cur.x);
  const uint32_t pw = cur.x - base_w;  // payload words of the tile before this chunk
  if (lane == 0) {
    uint32_t *tt = reinterpret_cast<uint32_t *>(out + 16 + 12 * (uint64_t)tile);
    tt[0] = cur.x - a.x;
    tt[1] = cur.y - a.y;
    tt[2] = cur.z - a.z;
  }
  if (on) {
    out[A + c0 + lane] = (uint8_t)(cc.x | (cc.y ? 0x80u : 0u));
    if (cc.y) {
      uint32_t *m = reinterpret_cast<uint32_t *>(out + Moff + 8 * (uint64_t)(cur.y - a.y));
      m[0] = (uint32_t)em;
      m[1] = (uint32_t)(em >> 32);
    }
    for (uint32_t k = 0; k < cc.x; k++) s_src[pw + k] = (uint16_t)(lane * 16 + k);
  }
  const uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int)(pw + cc.x), (int)tn - 1);  // payload words of the tile
  const uint32_t base = cur.x - a.x;                            // (lane 0's) before the tile
  const uint32_t base0 = __builtin_amdgcn_readfirstlane(base);
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
  // payload: 8-byte words of the tile in stream order
  const unsigned long long *__restrict__ pay = reinterpret_cast<const unsigned long long *>(P.pay);
  unsigned long long *__restrict__ dst = reinterpret_cast<unsigned long long *>(out + Poff) + base0;
  const unsigned long long *__restrict__ pays = pay + slot0 * 16;
  // (kPackUnroll words per lane in flight: every lane loads a clamped index
  // and only the words inside the tile are stored)
  for (uint32_t u0 = (uint32_t)lane; u0 < tot; u0 += kPackUnroll * kWave) {
    unsigned long long v[kPackUnroll];
#pragma unroll
    for (int j = 0; j < kPackUnroll; j++) v[j] = pays[s_src[min(u0 + (uint32_t)j * kWave, tot - 1)]];
#pragma unroll
    for (int j = 0; j < kPackUnroll; j++)
      if (u0 + (uint32_t)j * kWave < tot) dst[u0 + (uint32_t)j * kWave] = v[j];
  }
  // exact values of the chunks that have any, one chunk at a time
  const uint32_t *__restrict__ exv = reinterpret_cast<const uint32_t *>(P.exv);
  uint32_t *xo = reinterpret_cast<uint32_t *>(out + Xoff);
  const uint32_t px = cur.z - a.z;
  unsigned long long mx = __ballot(on && cc.z > 0);
  while (mx) {
    const int c = __builtin_ctzll(mx);
    mx &= mx - 1;
    const uint32_t nx = (uint32_t)__builtin_amdgcn_readlane((int)cc.z, c);
    const uint32_t pxc = (uint32_t)__builtin_amdgcn_readlane((int)px, c);
    if (__builtin_amdgcn_readlane((int)cc.w, c)) {
      // stored at their lanes: lane i's value is the popcount(mask below i)-th
      const unsigned long long emc =
          ((unsigned long long)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(em >> 32), c) << 32) |
          (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)em, c);
      if ((emc >> lane) & 1ull) xo[pxc + lanes_below(emc)] = exv[(slot0 + c) * 64 + lane];
    } else if ((uint32_t)lane < nx) {
      xo[pxc + lane] = exv[(slot0 + c) * 64 + lane];
    }
  }
}

__device__ inline uint32_t get32(const EncPlan &P, uint64_t off) {
  return *reinterpret_cast<const uint32_t *>(P.out + off);
}

template <int BS>
__device__ uint32_t block_sum(uint32_t v) {
  __shared__ uint32_t red[BS / kWave];
  v = wave_sum_u(v);
  if (lane_id() == 0) red[threadIdx.x / kWave] = v;
  __syncthreads();
  uint32_t t = 0;
  for (int i = 0; i < BS / kWave; i++) t += red[i];
  __syncthreads();
  return t;
}

// Block table: folds the block's workgroup records (min/max of the
// reconstructed values, input range, counts) and checksums its byte range.
// Partial checksums of the blocks' byte ranges: workgroup (b, seg) sums the
// words of its share of block b's sections, 8 bytes per thread and load.
// This workgroup's share (segment seg of kSumSegs) of the checksum of the
// 8-byte aligned byte range [start, end) of the stream, end - start a multiple
// of 8; word indices count from start.
__device__ uint32_t range_sum(const EncPlan &P, uint64_t start, uint64_t end, uint32_t seg) {
  uint32_t sum = 0;
  const uint32_t npair = (uint32_t)((end - start) / 8);
  const uint32_t per = (npair + kSumSegs - 1) / kSumSegs;
  const uint32_t lo = min(npair, seg * per), hi = min(npair, lo + per);
  const uint2 *__restrict__ src = reinterpret_cast<const uint2 *>(P.out + start);
  // four words per thread in flight (clamped loads; the sum wraps, so the
  // order of the terms does not change it)
  for (uint32_t i0 = lo + threadIdx.x; i0 < hi; i0 += 4 * kBS) {
    uint2 v[4];
#pragma unroll
    for (int j = 0; j < 4; j++) v[j] = src[min(i0 + (uint32_t)j * kBS, hi - 1)];
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const uint32_t i = i0 + (uint32_t)j * kBS;
      const uint32_t h = fmix32(v[j].x ^ (2u * i) * 0x9E3779B9u) + fmix32(v[j].y ^ (2u * i + 1u) * 0x9E3779B9u);
      sum += i < hi ? h : 0u;
    }
  }
  return block_sum<kBS>(sum);
}

__global__ __launch_bounds__(kBS) void k_block_sum(EncPlan P) {
  const Geo &g = P.g;
  const uint32_t b = blockIdx.x / kSumSegs, seg = blockIdx.x % kSumSegs;
  const uint64_t total = P.payload_off + P.secoff[g.nblocks * g.nL];
  const uint64_t start = P.payload_off + P.secoff[(int64_t)b * g.nL];
  const uint64_t end = P.payload_off + P.secoff[(int64_t)(b + 1) * g.nL];
  const uint32_t sum = total <= P.cap ? range_sum(P, start, end, seg) : 0u;
  if (threadIdx.x == 0) P.csum[blockIdx.x] = sum;
}

// Partial checksums of the section and block tables (after the block table
// is written), into the kSumSegs slots after the blocks' partials.
__global__ __launch_bounds__(kBS) void k_table_sum(EncPlan P) {
  const Geo &g = P.g;
  const uint64_t total = P.payload_off + P.secoff[g.nblocks * g.nL];
  const uint32_t sum = total <= P.cap ? range_sum(P, kHeaderBytes, P.payload_off, blockIdx.x) : 0u;
  if (threadIdx.x == 0) P.csum[g.nblocks * kSumSegs + blockIdx.x] = sum;
}

__global__ __launch_bounds__(kBS) void k_block_table(EncPlan P) {
  const Geo &g = P.g;
  const int64_t b = blockIdx.x;
  uint32_t sum = 0;
  for (int sgm = 0; sgm < kSumSegs; sgm++) sum += P.csum[b * kSumSegs + sgm];
  Part acc;
  part_init(acc);
  const Part *rec = P.part + b * P.part_per_block;
  const int L = g.nL - 1;
  for (int64_t i = threadIdx.x; i < P.part_per_block; i += kBS) {
    // records exist for level-0 workgroups, level-1 workgroups (nL >= 2),
    // level-2 workgroups (when level 2 has its own kernel) and the
    // coarse-level workgroup (nL >= 3)
    if (i == P.part_per_block - 1 && L < 2) continue;
    if (i >= P.part_l1 && i < P.part_l2 && L < 1) continue;
    if (i >= P.part_l2 && i < P.part_per_block - 1 && !P.l2fast) continue;
    const Part r = rec[i];
    acc.rmin = min(acc.rmin, r.rmin); acc.rmax = max(acc.rmax, r.rmax);
    acc.xmin = min(acc.xmin, r.xmin); acc.xmax = max(acc.xmax, r.xmax);
    acc.nonfinite |= r.nonfinite; acc.nO += r.nO; acc.nC += r.nC;
  }
  part_store(acc, &P.bst[b]);
  __syncthreads();
  if (threadIdx.x == 0) {
    const Part t = P.bst[b];
    const uint64_t bt = kHeaderBytes + 16 * (uint64_t)g.nblocks * g.nL + 16 * (uint64_t)b;
    put32(P, bt, __float_as_uint(of_ord(t.rmin)));
    put32(P, bt + 4, __float_as_uint(of_ord(t.rmax)));
    put32(P, bt + 8, sum);
    put32(P, bt + 12, g.diff ? P.act[b] : 0u);   // bit 0: active block (differentiated error control)
  }
}

struct ResultDev {
  uint64_t stream_bytes, n_outlier, n_corrected;
  int32_t status;
  float vmin, vmax;
  uint32_t reserved;
};

// Stream header, table checksum, header checksum, and the result record.
__device__ void header_words(const EncPlan &P, uint64_t total, bool fits, uint32_t sum, uint32_t (*red)[3],
                             unsigned long long (*redc)[2], uint32_t *hdr);

__global__ __launch_bounds__(kBS) void k_header(EncPlan P) {
  __shared__ uint32_t red[kWaves][3];
  __shared__ unsigned long long redc[kWaves][2];
  __shared__ uint32_t hdr[kHeaderBytes / 4];
  const Geo &g = P.g;
  const uint64_t total = P.payload_off + P.secoff[g.nblocks * g.nL];
  const bool fits = total <= P.cap;
  uint32_t xmin = 0xffffffffu, xmax = 0u, nf = 0u;
  unsigned long long nO = 0, nC = 0;
  for (int64_t b = threadIdx.x; b < g.nblocks; b += kBS) {
    const Part t = P.bst[b];
    xmin = min(xmin, t.xmin); xmax = max(xmax, t.xmax); nf |= t.nonfinite;
    nO += t.nO; nC += t.nC;
  }
  xmin = wave_min_u(xmin); xmax = wave_max_u(xmax); nf = wave_or(nf);
  for (int m = 32; m >= 1; m >>= 1) { nO += __shfl_xor(nO, m, kWave); nC += __shfl_xor(nC, m, kWave); }
  if (lane_id() == 0) {
    red[threadIdx.x / kWave][0] = xmin; red[threadIdx.x / kWave][1] = xmax; red[threadIdx.x / kWave][2] = nf;
    redc[threadIdx.x / kWave][0] = nO; redc[threadIdx.x / kWave][1] = nC;
  }
  __syncthreads();
  uint32_t sum = 0;
  for (int sgm = 0; sgm < kSumSegs; sgm++) sum += P.csum[g.nblocks * kSumSegs + sgm];
  if (threadIdx.x == 0) header_words(P, total, fits, sum, red, redc, hdr);
  __syncthreads();
  if (fits && threadIdx.x < kHeaderBytes / 4) put32(P, 4 * threadIdx.x, hdr[threadIdx.x]);
}

// Thread 0 of k_header: the header words and the compression result.
__device__ void header_words(const EncPlan &P, uint64_t total, bool fits, uint32_t sum, uint32_t (*red)[3],
                             unsigned long long (*redc)[2], uint32_t *hdr) {
  const Geo &g = P.g;
  for (int i = 1; i < kWaves; i++) {
    red[0][0] = min(red[0][0], red[i][0]); red[0][1] = max(red[0][1], red[i][1]); red[0][2] |= red[i][2];
    redc[0][0] += redc[i][0]; redc[0][1] += redc[i][1];
  }
  const float vmin = of_ord(red[0][0]), vmax = of_ord(red[0][1]);
  if (fits) {
    // the header's words in LDS and its checksum from them; the workgroup
    // writes them out together
    uint32_t *h = hdr;
    for (int i = 0; i < kHeaderBytes / 4; i++) h[i] = 0u;
    auto h64 = [&](int off, uint64_t v) {
      h[off / 4] = (uint32_t)v;
      h[off / 4 + 1] = (uint32_t)(v >> 32);
    };
    h[0] = kMagic;
    h[1] = kVersion;
    for (int a = 0; a < 3; a++) h64(8 + 8 * a, (uint64_t)g.n[a]);
    h[32 / 4] = (uint32_t)g.nL;
    h[36 / 4] = (uint32_t)g.B;
    h[40 / 4] = (uint32_t)g.qmax;
    h[44 / 4] = (uint32_t)g.K;
    uint64_t eb;
    __builtin_memcpy(&eb, &g.e, 8);
    h64(48, eb);
    h[56 / 4] = __float_as_uint(g.inv);
    h[60 / 4] = __float_as_uint(g.step);
    for (int j = 0; j < kMaxIso; j++) h[(64 + 4 * j) / 4] = __float_as_uint(j < g.K ? g.iso[j] : 0.0f);
    h[128 / 4] = __float_as_uint(vmin);
    h[132 / 4] = __float_as_uint(vmax);
    h64(136, (uint64_t)g.nblocks);
    for (int a = 0; a < 3; a++) h[(144 + 4 * a) / 4] = (uint32_t)g.nb[a];
    h[156 / 4] = (g.lossless ? 1u : 0u) | (g.diff ? 2u : 0u) | (g.diff && g.lossless2 ? 4u : 0u) |
                 (g.units ? 8u : 0u);
    h64(160, total);
    h64(168, redc[0][0]);
    h64(176, redc[0][1]);
    h64(184, P.payload_off);
    if (g.diff) {
      uint64_t e2;
      __builtin_memcpy(&e2, &g.e2, 8);
      h64(192, e2);
      h[200 / 4] = __float_as_uint(g.inv2);
      h[204 / 4] = __float_as_uint(g.step2);
    }
    if (g.units) {
      h[208 / 4] = (uint32_t)g.merge;
      for (int a = 0; a < 3; a++) h[(212 + 4 * a) / 4] = (uint32_t)g.mb[a];
    }
    h[248 / 4] = sum;
    uint32_t hs = 0;
    for (uint32_t j = 0; j < 63; j++) hs += fmix32(h[j] ^ (j * 0x9E3779B9u));
    h[252 / 4] = hs;
  }
  ResultDev *r = reinterpret_cast<ResultDev *>(P.result);
  r->stream_bytes = total;
  r->n_outlier = redc[0][0];
  r->n_corrected = redc[0][1];
  r->status = red[0][2] ? -1 : (fits ? 0 : -5);
  r->vmin = vmin;
  r->vmax = vmax;
  r->reserved = 0;
}

}  // namespace

int64_t encode_fine_groups(const EncPlan &p) {
  return p.tile0 ? encode_tile0_groups(p) : ceil_div(p.maxch[0], (int64_t)kWaves * p.cpw0);
}
int64_t encode_tile0_groups(const EncPlan &p) { return (p.g.B + 2) / 2; }
int64_t encode_l1_groups(const EncPlan &p) {
  if (p.tile1) return (p.g.B / 2 + 2) / 2;     // pairs of level-1 planes of a 64-cell block
  return p.g.nL >= 2 ? ceil_div(p.maxch[1] > 0 ? p.maxch[1] : 1, (int64_t)kChunksPerWG) : 0;
}
int64_t encode_l2_groups(const EncPlan &p) {
  if (p.top) return 0;                         // levels L .. 2 in one workgroup per block
  return p.g.nL >= 4 ? ceil_div(p.maxch[2] > 0 ? p.maxch[2] : 1, (int64_t)kChunksPerWG) : 0;
}

// A block's slab of planes spans < 4 GiB (the specialized kernels' 32-bit offsets).
static bool slab32(const Geo &g) {
  int64_t o[3], hi[3];
  largest_ext(g, o, hi);
  return 4.0 * (double)(hi[0] - o[0] + 1) * (double)g.n[1] * (double)g.n[2] < 4294967296.0;
}

bool encode_l2_fast(const EncPlan &p) { return !p.top && p.g.nL >= 4 && slab32(p.g) && p.l0.small; }

// Level 0 by plane pairs: 64-cell blocks below a coarser level, one
// quantizer, no per-point outputs, 32-bit offsets within a block's slab.
bool encode_tile0_ok(const EncPlan &p) {
  return p.g.B == 64 && p.g.nL >= 2 && !p.g.diff && !p.codes && !p.flags && slab32(p.g) && p.l0.small;
}

// Level 1 by plane pairs likewise, below a coarser level (level 2 exists).
bool encode_tile1_ok(const EncPlan &p) { return encode_tile0_ok(p) && p.g.nL >= 3; }

// Levels L .. 2 of a 64-cell block in one workgroup (level 2 exists).
bool encode_top_ok(const EncPlan &p) { return encode_tile1_ok(p); }

void encode_pack_layout(EncPlan &p) {
  const int L = p.g.nL - 1;
  int64_t base = 0;
  for (int l = L; l >= 0; l--) {
    p.pack_base[l] = base;
    p.pack_gpb[l] = ceil_div(p.maxch[l] > 0 ? p.maxch[l] : 1, (int64_t)64);  // tiles of 64 chunks
    base += p.g.nblocks * p.pack_gpb[l];
  }
  for (int l = L + 1; l < kMaxLevels; l++) { p.pack_base[l] = base; p.pack_gpb[l] = 1; }
}

template <int KB, bool DIFF>
void launch_encode_levels(const EncPlan &p, hipStream_t s) {
  const Geo &g = p.g;
  const int L = g.nL - 1;
  const int64_t gx = encode_fine_groups(p);
  if (L >= 2 && p.top) {
    prof_mark("k_encode_coarse", s, 0);
    k_encode_top<KB><<<dim3((unsigned)g.nblocks), dim3(kTopBS), 0, s>>>(p);
    prof_mark("k_encode_coarse", s, 1);
  } else if (L >= 2) {
    prof_mark("k_encode_coarse", s, 0);
    k_encode_coarse<KB><<<dim3((unsigned)g.nblocks), dim3(kBS), 0, s>>>(p, p.l2fast ? 3 : 2);
    if (p.l2fast) {
      const dim3 grid2((unsigned)encode_l2_groups(p), (unsigned)g.nblocks);
      if (!p.codes && !p.flags) k_encode_l2s<false, KB, 4, DIFF><<<grid2, dim3(kBS), 0, s>>>(p);
      else k_encode_l2s<true, KB, 1, DIFF><<<grid2, dim3(kBS), 0, s>>>(p);
    }
    prof_mark("k_encode_coarse", s, 1);
  }
  // the specialized kernels: 32-bit offsets within a block's slab and the
  // full-rate index arithmetic of small block shapes
  const bool fast = slab32(g) && p.l0.small;
  if (L >= 1) {
    const dim3 grid1((unsigned)encode_l1_groups(p), (unsigned)g.nblocks);
    prof_mark("k_encode_l1", s, 0);
    if (p.tile1) {
      if (g.lossless) k_encode_l1t<KB, true><<<grid1, dim3(kBS), 0, s>>>(p);
      else k_encode_l1t<KB, false><<<grid1, dim3(kBS), 0, s>>>(p);
    } else if (L >= 2 && fast && !p.codes && !p.flags)
      k_encode_l1s<false, KB, 4, DIFF><<<grid1, dim3(kBS), 0, s>>>(p);
    else if (L >= 2 && fast)
      k_encode_l1s<true, KB, 1, DIFF><<<grid1, dim3(kBS), 0, s>>>(p);
    else
      k_encode_l1<KB><<<grid1, dim3(kBS), 0, s>>>(p);
    prof_mark("k_encode_l1", s, 1);
  }
  if (gx > 0) {
    prof_mark("k_encode_fine", s, 0);
    const dim3 grid0((unsigned)gx, (unsigned)g.nblocks);
    if (p.tile0) {
      if (g.lossless) k_encode_l0t<KB, true><<<grid0, dim3(kBS), 0, s>>>(p);
      else k_encode_l0t<KB, false><<<grid0, dim3(kBS), 0, s>>>(p);
    } else if (L >= 1 && fast && !p.codes && !p.flags) {
      if (p.cpw0 % 4 == 0) k_encode_l0<false, KB, 4, DIFF><<<grid0, dim3(kBS), 0, s>>>(p);
      else if (p.cpw0 % 2 == 0) k_encode_l0<false, KB, 2, DIFF><<<grid0, dim3(kBS), 0, s>>>(p);
      else k_encode_l0<false, KB, 1, DIFF><<<grid0, dim3(kBS), 0, s>>>(p);
    } else if (L >= 1 && fast) {
      k_encode_l0<true, KB, 1, DIFF><<<grid0, dim3(kBS), 0, s>>>(p);
    } else {
      k_encode_fine<KB><<<grid0, dim3(kBS), 0, s>>>(p);
    }
    prof_mark("k_encode_fine", s, 1);
  }
}

// Index signatures of the blocks (block merging before compression): the
// input's min and max per closed block extent, then one signature word per
// block in p.act[0 .. nblocks).
void launch_block_signatures(const EncPlan &p, hipStream_t s) {
  const Geo &g = p.g;
  k_block_minmax<<<dim3((unsigned)kActSplit, (unsigned)g.nblocks), dim3(kBS), 0, s>>>(p);
  k_block_sig<<<dim3((unsigned)ceil_div(g.nblocks, kBS)), dim3(kBS), 0, s>>>(p);
}

void launch_encode(const EncPlan &p, int64_t, U4 *scan_tmp, uint64_t *scan_tmp64, hipStream_t s) {
  const Geo &g = p.g;
  const int64_t nsec = g.nblocks * g.nL;
  if (g.diff) {
    // block activity on the input (closed extents) for the per-point quantizer choice
    k_block_minmax<<<dim3((unsigned)kActSplit, (unsigned)g.nblocks), dim3(kBS), 0, s>>>(p);
    k_block_active_final<<<dim3((unsigned)ceil_div(g.nblocks, kBS)), dim3(kBS), 0, s>>>(p);
    if (g.K <= 1) launch_encode_levels<1, true>(p, s);
    else if (g.K <= 2) launch_encode_levels<2, true>(p, s);
    else if (g.K <= 4) launch_encode_levels<4, true>(p, s);
    else launch_encode_levels<16, true>(p, s);
  } else {
    if (g.K <= 1) launch_encode_levels<1, false>(p, s);
    else if (g.K <= 2) launch_encode_levels<2, false>(p, s);
    else if (g.K <= 4) launch_encode_levels<4, false>(p, s);
    else launch_encode_levels<16, false>(p, s);
  }
  scan_u4(p.cnt, p.P, p.nslots, scan_tmp, s);
  prof_mark("k_sections", s, 0);
  k_sections<<<dim3((unsigned)ceil_div(nsec, kBS)), dim3(kBS), 0, s>>>(p);
  prof_mark("k_sections", s, 1);
  scan_u64(p.secsz, p.secoff, nsec, scan_tmp64, s);
  prof_mark("k_sec_table", s, 0);
  k_sec_table<<<dim3((unsigned)ceil_div(nsec, kBS)), dim3(kBS), 0, s>>>(p);
  prof_mark("k_sec_table", s, 1);
  const int64_t npack = p.pack_base[0] + g.nblocks * p.pack_gpb[0];
  if (p.nslots > 0 && npack > 0) {
    prof_mark("k_pack", s, 0);
    k_pack<<<dim3((unsigned)ceil_div(npack, kWaves)), dim3(kBS), 0, s>>>(p);
    prof_mark("k_pack", s, 1);
  }
  prof_mark("k_block_table", s, 0);
  k_block_sum<<<dim3((unsigned)(g.nblocks * kSumSegs)), dim3(kBS), 0, s>>>(p);
  k_block_table<<<dim3((unsigned)g.nblocks), dim3(kBS), 0, s>>>(p);
  if (g.units) k_box_table<<<dim3((unsigned)ceil_div(8 * g.nblocks, kBS)), dim3(kBS), 0, s>>>(p);
  k_table_sum<<<dim3((unsigned)kSumSegs), dim3(kBS), 0, s>>>(p);
  prof_mark("k_block_table", s, 1);
  prof_mark("k_header", s, 0);
  k_header<<<dim3(1), dim3(kBS), 0, s>>>(p);
  prof_mark("k_header", s, 1);
}

}  // namespace chr
