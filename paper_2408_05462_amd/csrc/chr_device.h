// chr_device.h -- shared definitions of the gfx950 CHR kernels.
//
// Stream format (little-endian; all offsets in bytes from the stream start):
//   header, 256 bytes:
//     0 u32 magic "CHR1"   4 u32 version=1   8 i64 nz  16 i64 ny  24 i64 nx
//     32 i32 levels  36 i32 block  40 i32 qmax  44 i32 n_iso  48 f64 e
//     56 f32 1/(2e)  60 f32 2e  64 f32 iso[16]  128 f32 vmin  132 f32 vmax
//     136 i64 nblocks (storage units)  144 i32 nbz,nby,nbx (block grid)
//     156 u32 flags (bit0 lossless, bit1 differentiated bounds, bit2 far
//     bound lossless, bit3 merged units)  160 u64 total bytes
//     168 u64 #outliers  176 u64 #corrections  184 u64 payload offset
//     192 f64 far bound  200 f32 1/(2 e_far)  204 f32 2 e_far
//     208 u32 merge (largest blocks per axis of a unit)  212 u32 largest unit
//     extent in blocks along z, y, x  248 u32 table checksum
//     252 u32 header checksum
//   section table at 256: per unit (blocks bz,by,bx lexicographic, or the
//     merged units in order), per level from the coarsest: {u64 offset,
//     u64 bytes}
//   block table: per unit {f32 min, f32 max, u32 checksum, u32 activity}
//   box table (merged streams only): per unit {u32 first block z, y, x,
//     u32 one past the last block z, y, x, u32 0, u32 0}
//   payload: units in order, each the concatenation of its sections.
//   section (the points of one level in one closed block, lexicographic z,y,x):
//     u32 npts, u32 W, u32 NE, u32 NX
//     tile table: per 64 chunks {u32 W, u32 NE, u32 NX before the tile}, pad 8
//     chunk header bytes (bits 0-4 width w <= 16, bit 7 has exact values), pad 8
//     payload: per 64-point chunk w u64 words, code of lane i at bits [i*w,(i+1)*w)
//       (code = zigzag of the quantization code; 0 where stored exactly)
//     exact masks: u64 per chunk that has exact values (bit i = lane i)
//     exact values: binary32 bits in chunk order then lane order, pad 8
//   checksum of a byte range: sum mod 2^32 of fmix32(word_j ^ j*0x9E3779B9)
//     over its 32-bit words (fmix32 = MurmurHash3's finalizer).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace chr {

constexpr uint32_t kMagic = 0x31524843u;
constexpr uint32_t kVersion = 1u;
constexpr int kHeaderBytes = 256;
constexpr int kMaxIso = 16;
constexpr int kMaxW = 16;           // 32767 -> zigzag < 2^16
constexpr int kWave = 64;

// Everything a kernel needs to know about the field and the hierarchy.
struct Geo {
  int64_t n[3];      // dims z, y, x
  int64_t nb[3];     // blocks per axis
  int64_t nblocks;
  int nL, B, qmax, K;
  double e;
  float inv, step;
  int lossless;
  // a binary32 bound below e by more than the rounding of one binary32
  // subtraction: |fl(x' - x)| <= ein proves |x' - x| <= e exactly
  float ein;
  float iso[kMaxIso];
  // differentiated error control: points of no block crossing a candidate
  // isovalue use the far quantizer (diff = 0: one quantizer everywhere)
  double e2;
  float inv2, step2;
  int lossless2, diff;
  // block merging before compression: storage units are rectangles of
  // blocks, units[8u .. 8u+5] = first block and one past the last block of
  // unit u along z, y, x (device memory); nullptr: one unit per block, and
  // nblocks counts blocks.  merge: largest blocks per axis of a unit (1
  // without merging); mb: the largest unit extent in blocks.
  const uint32_t *units;
  int merge;
  int mb[3];
};

// The quantizer constants of one point.
struct QuantP {
  double e;
  float inv, step;
  int lossless;
};

__host__ __device__ inline QuantP quant_pick(const Geo &g, bool far) {
  QuantP q;
  q.e = far ? g.e2 : g.e;
  q.inv = far ? g.inv2 : g.inv;
  q.step = far ? g.step2 : g.step;
  q.lossless = far ? g.lossless2 : g.lossless;
  return q;
}

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

__host__ __device__ inline int64_t blocks_along(int64_t n, int64_t B) {
  return n - 1 <= 0 ? 1 : ceil_div(n - 1, B);
}

// Closed extent [o, hi] of block b (lexicographic bz, by, bx).
__host__ __device__ inline void block_ext(const Geo &g, int64_t b, int64_t o[3], int64_t hi[3]);

// Closed extent of storage unit b: block b, or merged unit b (its box read
// from the unit table, clamped to the block grid so that a corrupt table
// cannot reach outside the field).
__device__ inline void unit_ext(const Geo &g, int64_t b, int64_t o[3], int64_t hi[3]) {
  if (!g.units) {
    block_ext(g, b, o, hi);
    return;
  }
  const uint32_t *e = g.units + 8 * b;
  for (int a = 0; a < 3; a++) {
    int64_t b1 = (int64_t)e[3 + a];
    b1 = b1 < 1 ? 1 : (b1 > g.nb[a] ? g.nb[a] : b1);
    const int64_t b0 = (int64_t)e[a] < b1 - 1 ? (int64_t)e[a] : b1 - 1;
    const int64_t h = b1 * (int64_t)g.B;
    o[a] = b0 * g.B;
    hi[a] = h < g.n[a] - 1 ? h : g.n[a] - 1;
  }
}

// The extent of the largest storage unit (its origin at 0): block 0, or a
// unit of mb blocks per axis.  Host code sizes launches with it.
__host__ __device__ inline void largest_ext(const Geo &g, int64_t o[3], int64_t hi[3]) {
  for (int a = 0; a < 3; a++) {
    const int64_t e = (int64_t)(g.merge > 1 ? g.mb[a] : 1) * g.B;
    o[a] = 0;
    hi[a] = e < g.n[a] - 1 ? e : g.n[a] - 1;
  }
}

__host__ __device__ inline void block_ext(const Geo &g, int64_t b, int64_t o[3], int64_t hi[3]) {
  int64_t bi[3];
  bi[2] = b % g.nb[2];
  bi[1] = (b / g.nb[2]) % g.nb[1];
  bi[0] = b / (g.nb[2] * g.nb[1]);
  for (int a = 0; a < 3; a++) {
    o[a] = bi[a] * g.B;
    hi[a] = o[a] + g.B;
    if (hi[a] > g.n[a] - 1) hi[a] = g.n[a] - 1;
  }
}

// Differentiated error control (Sec. II.A: blocks with different error
// bounds).  A block is active when the input on its closed extent crosses a
// candidate isovalue; a point takes the near bound when any block whose
// closed extent contains it is active.  A point shared by blocks so gets one
// bound, hence one value, in all of them.  Block b's points fall in 27
// position classes: per axis 0 on the face shared with the lower neighbour,
// 2 on the face shared with the upper one, 1 otherwise; bit 9cz + 3cy + cx
// of `lut` tells whether the class takes the near bound.
constexpr uint32_t kNearAll = (1u << 27) - 1u;   // every class near

struct NearSel {
  uint32_t lut;
  uint32_t lo[3], hi[3];   // coordinates of the shared faces (0xffffffff: no neighbour)
};

// act[i * stride] bit 0: block i is active.  Every lane of the wave takes
// part (two ballots); lane t < 27 looks at neighbour t, then at class t.
__device__ inline NearSel near_sel(const Geo &g, const uint32_t *act, uint32_t stride, int64_t b,
                                   const int64_t o[3], const int64_t hi[3]) {
  const int64_t bi[3] = {b / (g.nb[2] * g.nb[1]), (b / g.nb[2]) % g.nb[1], b % g.nb[2]};
  const int lane = (int)__lane_id();
  bool a = false;
  if (lane < 27) {
    const int64_t nz = bi[0] + lane / 9 - 1, ny = bi[1] + (lane / 3) % 3 - 1, nx = bi[2] + lane % 3 - 1;
    if (nz >= 0 && nz < g.nb[0] && ny >= 0 && ny < g.nb[1] && nx >= 0 && nx < g.nb[2])
      a = (act[(uint64_t)((nz * g.nb[1] + ny) * g.nb[2] + nx) * stride] & 1u) != 0;
  }
  const uint64_t M = __ballot(a);
  bool nr = false;
  if (lane < 27) {
    // the blocks holding a point of class (cz, cy, cx): offsets {0, c - 1} per axis
    const int cz = lane / 9, cy = (lane / 3) % 3, cx = lane % 3;
    for (int dz = min(cz - 1, 0); dz <= max(cz - 1, 0); dz++)
      for (int dy = min(cy - 1, 0); dy <= max(cy - 1, 0); dy++)
        for (int dx = min(cx - 1, 0); dx <= max(cx - 1, 0); dx++)
          nr |= ((M >> ((dz + 1) * 9 + (dy + 1) * 3 + (dx + 1))) & 1ull) != 0;
  }
  NearSel s;
  s.lut = (uint32_t)__ballot(nr);
  for (int ax = 0; ax < 3; ax++) {
    s.lo[ax] = bi[ax] > 0 ? (uint32_t)o[ax] : 0xffffffffu;
    s.hi[ax] = bi[ax] + 1 < g.nb[ax] ? (uint32_t)hi[ax] : 0xffffffffu;
  }
  return s;
}

__device__ inline bool near_at(const NearSel &s, uint32_t z, uint32_t y, uint32_t x) {
  const uint32_t cz = z == s.lo[0] ? 0u : (z == s.hi[0] ? 2u : 1u);
  const uint32_t cy = y == s.lo[1] ? 0u : (y == s.hi[1] ? 2u : 1u);
  const uint32_t cx = x == s.lo[2] ? 0u : (x == s.hi[2] ? 2u : 1u);
  return ((s.lut >> (cz * 9u + cy * 3u + cx)) & 1u) != 0;
}

// Division by a runtime constant d for dividends below 2^31: with
// l = ceil(log2 d) and m = floor(2^(31+l)/d) + 1 (< 2^32), n/d equals
// mulhi(n, m) >> (l-1) for every n < 2^31 (Granlund-Montgomery).
struct FastDiv {
  uint32_t d, m;
  uint32_t sh;    // l - 1 (0 when d == 1)
  uint32_t one;   // d == 1: the quotient is n itself
};

__host__ __device__ inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  int l = 0;
  while (((uint64_t)1 << l) < (uint64_t)d) l++;
  if (l == 0) {
    f.m = 0;
    f.sh = 0;
    f.one = 1;
  } else {
    f.m = (uint32_t)((((uint64_t)1) << (31 + l)) / d + 1);
    f.sh = (uint32_t)(l - 1);
    f.one = 0;
  }
  return f;
}

// Branch-free: one multiply-high, one shift, one select.
__host__ __device__ inline uint32_t fdiv(uint32_t n, const FastDiv &f) {
#ifdef __HIP_DEVICE_COMPILE__
  const uint32_t q = __umulhi(n, f.m) >> f.sh;
#else
  const uint32_t q = (uint32_t)(((uint64_t)n * f.m) >> 32) >> f.sh;
#endif
  return f.one ? n : q;
}

// Level-l section of one closed block: the points of the block's 2^l grid
// that are not on its 2^(l+1) grid (all of them at the top level), visited in
// lexicographic (z, y, x) order.  Local grid index (w, v, u) -> coordinate
// o + (w, v, u) * 2^l.
struct Sec {
  uint32_t mx, my, mz;   // 2^l-grid points per axis in the block
  uint32_t rowE;         // points in an even row of an even plane (odd u)
  uint32_t Pe, Po;       // points in an even / odd plane
  uint32_t npts;
  int top;
  FastDiv d_pair, d_rp, d_mx, d_my;
};

__host__ __device__ inline Sec sec_geom(const int64_t o[3], const int64_t hi[3], int l, int L) {
  Sec s;
  s.mz = (uint32_t)((hi[0] - o[0]) >> l) + 1;
  s.my = (uint32_t)((hi[1] - o[1]) >> l) + 1;
  s.mx = (uint32_t)((hi[2] - o[2]) >> l) + 1;
  s.top = (l == L);
  if (s.top) {
    s.rowE = 0; s.Pe = 0; s.Po = s.mx * s.my;
    s.npts = s.mx * s.my * s.mz;
  } else {
    uint32_t cx = (s.mx + 1) / 2, cy = (s.my + 1) / 2, cz = (s.mz + 1) / 2;
    s.rowE = s.mx - cx;
    s.Pe = s.my * s.mx - cy * cx;
    s.Po = s.my * s.mx;
    s.npts = s.mz * s.my * s.mx - cz * cy * cx;
  }
  s.d_pair = make_fastdiv(s.Pe + s.Po);
  s.d_rp = make_fastdiv(s.rowE + s.mx);
  s.d_mx = make_fastdiv(s.mx);
  s.d_my = make_fastdiv(s.my);
  return s;
}

__host__ __device__ inline void sec_point(const Sec &s, uint32_t j, uint32_t &w, uint32_t &v, uint32_t &u) {
  if (s.top) {
    const uint32_t t = fdiv(j, s.d_mx);
    u = j - t * s.mx;
    w = fdiv(t, s.d_my);
    v = t - w * s.my;
    return;
  }
  const uint32_t pair = s.Pe + s.Po;
  const uint32_t w2 = fdiv(j, s.d_pair);
  uint32_t r = j - w2 * pair;
  if (r < s.Pe) {
    w = 2 * w2;
    const uint32_t RP = s.rowE + s.mx;
    const uint32_t v2 = fdiv(r, s.d_rp), t = r - v2 * RP;
    if (t < s.rowE) { v = 2 * v2; u = 2 * t + 1; }
    else { v = 2 * v2 + 1; u = t - s.rowE; }
  } else {
    r -= s.Pe;
    w = 2 * w2 + 1;
    v = fdiv(r, s.d_mx);
    u = r - v * s.mx;
  }
}

// Division by a block-shape constant d without 32-bit multiplies: with r the
// smallest binary32 value >= 1/d, trunc(fl(n * r)) equals floor(n / d) for
// every n, d < 2^21.  (n * r exceeds n/d by at most n/d * 2^-23 and rounding
// adds at most half an ulp of a value below 2^21/d + 1, so the result stays
// below the next integer, whose distance from n/d is at least 1/d; it never
// drops below floor(n/d), which is representable.)
struct SecR {
  float r_pair, r_rp, r_mx;  // reciprocals of Pe + Po, rowE + mx and mx
};

__host__ inline float rcp_up(uint32_t d) {
  const double t = 1.0 / (double)d;
  float r = (float)t;
  if ((double)r < t) r = nextafterf(r, 3.0e38f);
  return r;
}

__host__ inline SecR sec_rcp(const Sec &s) {
  SecR r;
  r.r_pair = rcp_up(s.Pe + s.Po);
  r.r_rp = rcp_up(s.rowE + s.mx);
  r.r_mx = rcp_up(s.mx);
  return r;
}

__device__ inline uint32_t qdiv(uint32_t n, float r) { return (uint32_t)__fmul_rn((float)n, r); }

// 24-bit multiplies (operands < 2^24, low 32 bits of the product) in one
// full-rate instruction each; the compiler otherwise may fold the operand
// masks of __umul24 away and emit a quarter-rate 32-bit multiply.  `s`: the
// second operand is wave-uniform (a scalar register).
__device__ inline uint32_t mad24s(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t r;
  asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(b), "v"(c));
  return r;
}
__device__ inline uint32_t mul24s(uint32_t a, uint32_t b) {
  uint32_t r;
  asm("v_mul_u32_u24 %0, %1, %2" : "=v"(r) : "s"(b), "v"(a));
  return r;
}
__device__ inline uint32_t mul24v(uint32_t a, uint32_t b) {
  uint32_t r;
  asm("v_mul_u32_u24 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// sec_point for a section below the top level with npts < 2^21: full-rate
// arithmetic only (the reciprocal division above and 24-bit multiplies).
__device__ inline void sec_point24(const Sec &s, const SecR &rc, uint32_t j, uint32_t &w, uint32_t &v,
                                   uint32_t &u) {
  const uint32_t w2 = qdiv(j, rc.r_pair);
  const uint32_t r = j - mul24s(w2, s.Pe + s.Po);
  const bool ev = r < s.Pe;  // even plane: rows alternate odd-u-only and full
  const uint32_t n = ev ? r : r - s.Pe;
  const uint32_t q = qdiv(n, ev ? rc.r_rp : rc.r_mx);
  const uint32_t t = n - mul24v(q, ev ? s.rowE + s.mx : s.mx);
  const bool odd_only = ev && t < s.rowE;
  w = 2 * w2 + (ev ? 0u : 1u);
  v = ev ? 2 * q + (odd_only ? 0u : 1u) : q;
  u = odd_only ? 2 * t + 1 : (ev ? t - s.rowE : t);
}

__device__ inline float avg2(float a, float b) { return __fmul_rn(__fadd_rn(a, b), 0.5f); }

// Multilinear midpoint from the coarser compact grid, given the parent rows
// (za,ya), (za,yb), (zb,ya), (zb,yb) and x positions xa, xb: along each odd
// axis the two parents are averaged (xu, yu, zu false: the lower parent
// alone), first along x, then y, then z.  Every parent is loaded before any
// arithmetic, so the eight loads are in flight together instead of one
// dependent round trip per axis.
__device__ inline float midpoint8(float a0, float a1, float b0, float b1, float c0, float c1, float d0, float d1,
                                  bool zu, bool yu, bool xu) {
  const float A = xu ? avg2(a0, a1) : a0, B = xu ? avg2(b0, b1) : b0;
  const float Cz = xu ? avg2(c0, c1) : c0, D = xu ? avg2(d0, d1) : d0;
  const float p0 = yu ? avg2(A, B) : A;
  const float p1 = yu ? avg2(Cz, D) : Cz;
  return zu ? avg2(p0, p1) : p0;
}

__device__ inline float midpoint_rows(const float *__restrict__ r00, const float *__restrict__ r01,
                                      const float *__restrict__ r10, const float *__restrict__ r11, uint32_t xa,
                                      uint32_t xb, bool zu, bool yu, bool xu) {
  return midpoint8(r00[xa], r00[xb], r01[xa], r01[xb], r10[xa], r10[xb], r11[xa], r11[xb], zu, yu, xu);
}

// Holds a value in a register at this point of the program: the arithmetic
// that produces it stays above, instead of being moved into the branch that
// uses it (so every load it reads is waited for before any later store).
// v_writelane: lane L (wave-uniform, through M0) of dst takes the
// wave-uniform value v.
__device__ __forceinline__ void writelane(uint32_t &dst, uint32_t v, uint32_t L) {
  asm volatile("s_mov_b32 m0, %2\n\tv_writelane_b32 %0, %1, m0" : "+v"(dst) : "s"(v), "s"(L) : "m0");
}

__device__ inline void hold(float &v) { asm volatile("" : "+v"(v)); }
__device__ inline void hold(uint32_t &v) { asm volatile("" : "+v"(v)); }

// Load of a float at a 32-bit byte offset from a uniform base (lets the
// compiler use the scalar-base + 32-bit vector-offset addressing form).
__device__ inline float ldf(const char *__restrict__ base, uint32_t off) {
  return *reinterpret_cast<const float *>(base + off);
}
__device__ inline uint32_t ldu(const char *__restrict__ base, uint32_t off) {
  return *reinterpret_cast<const uint32_t *>(base + off);
}
__device__ inline void stf(char *__restrict__ base, uint32_t off, float v) {
  *reinterpret_cast<float *>(base + off) = v;
}
__device__ inline void stu(char *__restrict__ base, uint32_t off, uint32_t v) {
  *reinterpret_cast<uint32_t *>(base + off) = v;
}

// Level-0 section geometry of the (at most 8) block shapes -- interior or
// last block along each axis -- plus divisors that split a block index into
// (bz, by, bx); filled on the host so kernels skip the 64-bit arithmetic.
struct L0Geo {
  Sec sec[8];    // level 0
  Sec sec1[8];   // level 1 (when the hierarchy has one)
  Sec sec2[8];   // level 2 (when the hierarchy has one)
  SecR rc[8];    // level-0 reciprocals (valid when small)
  SecR rc1[8];   // level-1 reciprocals
  SecR rc2[8];   // level-2 reciprocals
  FastDiv d_nb2, d_nb1;
  uint32_t nb[3];
  int small;     // every level-0 section has < 2^21 points and the index
                 // products of the level-0 kernels stay below 2^24
};

__host__ inline void make_l0geo(const Geo &g, L0Geo &G) {
  for (int a = 0; a < 3; a++) G.nb[a] = (uint32_t)g.nb[a];
  G.d_nb2 = make_fastdiv(G.nb[2]);
  G.d_nb1 = make_fastdiv(G.nb[1]);
  for (int cls = 0; cls < 8; cls++) {
    const int64_t bz = (cls & 4) ? g.nb[0] - 1 : 0, by = (cls & 2) ? g.nb[1] - 1 : 0, bx = (cls & 1) ? g.nb[2] - 1 : 0;
    int64_t o[3], hi[3];
    block_ext(g, (bz * g.nb[1] + by) * g.nb[2] + bx, o, hi);
    G.sec[cls] = sec_geom(o, hi, 0, g.nL - 1);
    G.sec1[cls] = sec_geom(o, hi, g.nL >= 2 ? 1 : 0, g.nL - 1);
    G.sec2[cls] = sec_geom(o, hi, g.nL >= 3 ? 2 : 0, g.nL - 1);
    G.rc[cls] = sec_rcp(G.sec[cls]);
    G.rc1[cls] = sec_rcp(G.sec1[cls]);
    G.rc2[cls] = sec_rcp(G.sec2[cls]);
  }
  // row products w * n1 + y and plane offsets of the field and of the
  // level-1 grid within a block's slab, as 24-bit multiplier operands
  const int64_t lim = (int64_t)1 << 21, lim24 = (int64_t)1 << 24;
  int64_t maxpts = 0;
  for (int cls = 0; cls < 8; cls++) maxpts = maxpts > G.sec[cls].npts ? maxpts : G.sec[cls].npts;
  const int64_t n1 = g.n[1], n2 = g.n[2], g1 = (n1 + 1) / 2, g2 = (n2 + 1) / 2;
  G.small = maxpts < lim && (int64_t)(g.B + 1) * n1 < lim24 && n2 < lim24 &&
            (int64_t)(g.B / 2 + 2) * g1 < lim24 && g2 < lim24 && g.B + 1 < lim;
}

// Block b's origin, closed-extent end, first non-owned coordinate and shape class.
struct BlockPos {
  uint32_t o[3], hi[3], own[3];
  int cls;
};

__device__ inline BlockPos block_pos(const Geo &g, const L0Geo &G, uint32_t b) {
  BlockPos p;
  const uint32_t t = fdiv(b, G.d_nb2);
  const uint32_t bx = b - t * G.nb[2];
  const uint32_t bz = fdiv(t, G.d_nb1);
  const uint32_t by = t - bz * G.nb[1];
  const uint32_t bi[3] = {bz, by, bx};
  p.cls = 0;
  for (int a = 0; a < 3; a++) {
    const uint32_t n = (uint32_t)g.n[a];
    p.o[a] = bi[a] * (uint32_t)g.B;
    const uint32_t e = p.o[a] + (uint32_t)g.B;
    p.hi[a] = e < n - 1 ? e : n - 1;
    p.own[a] = e < n - 1 ? e : n;
    if (bi[a] == G.nb[a] - 1) p.cls |= 4 >> a;
  }
  return p;
}

// Levels L .. 2 of a 64-cell block (its points of the 4-grid, at most 17^3)
// in one 1024-thread workgroup, compression and reconstruction alike: each
// thread owns fixed 4-grid points, whose section indices follow in closed
// form from their coordinates.
constexpr int kTopSide = 17;                             // 4-grid points per axis of a 64-cell block
constexpr int kTopPts = kTopSide * kTopSide * kTopSide;  // 4913
constexpr int kTopCodes = kTopPts + 6 * 64;              // codes of every level (at most 5), each 64-aligned
constexpr int kTopBS = 1024;                             // threads per block
constexpr int kTopWaves = kTopBS / kWave;
constexpr int kTopPer = (kTopPts + kTopBS - 1) / kTopBS; // 4-grid points per thread

__device__ inline uint32_t top_idx(uint32_t z, uint32_t y, uint32_t x) { return (z * kTopSide + y) * kTopSide + x; }

// The section sizes of level l of a block (as sec_geom, without divisors).
struct SecDims {
  uint32_t mx, my, mz, rowE, Pe, Po, npts;
};
__device__ inline SecDims sec_dims(const BlockPos &bp, int l, int L) {
  SecDims d;
  d.mz = ((bp.hi[0] - bp.o[0]) >> l) + 1;
  d.my = ((bp.hi[1] - bp.o[1]) >> l) + 1;
  d.mx = ((bp.hi[2] - bp.o[2]) >> l) + 1;
  if (l == L) {
    d.rowE = 0; d.Pe = 0; d.Po = d.mx * d.my;
    d.npts = d.mx * d.my * d.mz;
  } else {
    const uint32_t cx = (d.mx + 1) / 2, cy = (d.my + 1) / 2, cz = (d.mz + 1) / 2;
    d.rowE = d.mx - cx;
    d.Pe = d.my * d.mx - cy * cx;
    d.Po = d.my * d.mx;
    d.npts = d.mz * d.my * d.mx - cz * cy * cx;
  }
  return d;
}

// Point i of a block's 4-grid (dims d0 x d1 x d2 <= 17^3) packed in one word:
// x, y, z (clamped into the block) in bits 0-4, 5-9, 10-14, and from bit 15
// the point's level + 1 (the fewest trailing zeros of its non-zero
// coordinates, plus 2, at most L), 0 for no point.
__device__ inline uint32_t top_point(uint32_t i, uint32_t d0, uint32_t d1, uint32_t d2, int L) {
  const uint32_t z = i / (kTopSide * kTopSide), y = (i / kTopSide) % kTopSide, x = i % kTopSide;
  const bool in = i < (uint32_t)kTopPts && z < d0 && y < d1 && x < d2;
  int lv = L;
  if (z) lv = min(lv, 2 + __builtin_ctz(z));
  if (y) lv = min(lv, 2 + __builtin_ctz(y));
  if (x) lv = min(lv, 2 + __builtin_ctz(x));
  const uint32_t zc = min(z, d0 - 1), yc = min(y, d1 - 1), xc = min(x, d2 - 1);
  return xc | (yc << 5) | (zc << 10) | (in ? (uint32_t)(lv + 1) << 15 : 0u);
}

// Section index of the level-l point (w, v, u) (level-l units): lexicographic
// over the level's points (the anchors' level: every point).
__device__ inline uint32_t sec_index(const SecDims &d, bool top, uint32_t w, uint32_t v, uint32_t u) {
  if (top) return (w * d.my + v) * d.mx + u;
  const uint32_t base = (w >> 1) * (d.Pe + d.Po);
  if (w & 1u) return base + d.Pe + v * d.mx + u;
  const uint32_t row = (v >> 1) * (d.rowE + d.mx);
  return (v & 1u) ? base + row + d.rowE + u : base + row + (u >> 1);
}

// Workgroups are dispatched to the 8 XCDs round-robin by linear id.  This
// maps linear id i of a 2D grid to logical work so that each XCD receives a
// contiguous eighth of the work (its L2 then sees neighbouring data).
__device__ inline void xcd_remap(uint32_t &bx, uint32_t &by) {
  const uint32_t gx = gridDim.x, n = gridDim.x * gridDim.y;
  const uint32_t i = blockIdx.y * gx + blockIdx.x;
  const uint32_t n8 = n >> 3;
  const uint32_t l = (i < (n8 << 3)) ? (i & 7u) * n8 + (i >> 3) : i;
  by = l / gx;
  bx = l - by * gx;
}

__host__ __device__ inline size_t pad8(size_t n) { return (n + 7) & ~(size_t)7; }

__host__ __device__ inline uint64_t sec_bytes(uint64_t npts, uint64_t W, uint64_t NE, uint64_t NX) {
  uint64_t nch = (npts + 63) / 64, ntile = (nch + 63) / 64;
  return 16 + pad8(12 * ntile) + pad8(nch) + 8 * W + 8 * NE + pad8(4 * NX);
}

// Compact grid of level l: the points whose coordinates are multiples of 2^l.
__host__ __device__ inline int64_t lvl_dim(int64_t n, int l) { return ((n - 1) >> l) + 1; }

// Ordered-integer image of a binary32 value: unsigned comparison of the
// images is the total order with -0 < +0.
__host__ __device__ inline uint32_t ord_of(float f) {
  uint32_t u;
  __builtin_memcpy(&u, &f, 4);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__host__ __device__ inline float of_ord(uint32_t o) {
  uint32_t u = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
  float f;
  __builtin_memcpy(&f, &u, 4);
  return f;
}

__host__ __device__ inline uint32_t fmix32(uint32_t h) {
  h ^= h >> 16; h *= 0x85ebca6bu; h ^= h >> 13; h *= 0xc2b2ae35u; h ^= h >> 16;
  return h;
}

// ---------------------------------------------------------------- waves

__device__ inline int lane_id() { return (int)__lane_id(); }

__device__ inline uint32_t wave_or(uint32_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v |= __shfl_xor(v, m, kWave);
  return v;
}
__device__ inline uint32_t wave_min_u(uint32_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) { uint32_t o = __shfl_xor(v, m, kWave); v = o < v ? o : v; }
  return v;
}
__device__ inline uint32_t wave_max_u(uint32_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) { uint32_t o = __shfl_xor(v, m, kWave); v = o > v ? o : v; }
  return v;
}
__device__ inline uint32_t wave_sum_u(uint32_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, kWave);
  return v;
}
// exclusive prefix sum over the lanes of a wave
__device__ inline uint32_t wave_excl_sum(uint32_t v) {
  uint32_t x = v;
  int lid = lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    uint32_t y = __shfl_up(x, d, kWave);
    if (lid >= d) x += y;
  }
  return x - v;
}
// Wave-wide reductions through DPP: within each 16-lane row (xor 1, xor 2,
// half mirror, mirror), then across rows (broadcast of lanes 15 and 31);
// lane 63 ends with the result, which is read back as a wave-uniform value.
template <class Op>
__device__ inline uint32_t wave_reduce_dpp(uint32_t v, Op op, uint32_t ident) {
  v = op(v, (uint32_t)__builtin_amdgcn_update_dpp((int)ident, (int)v, 0xb1, 0xf, 0xf, false));   // quad_perm 1,0,3,2
  v = op(v, (uint32_t)__builtin_amdgcn_update_dpp((int)ident, (int)v, 0x4e, 0xf, 0xf, false));   // quad_perm 2,3,0,1
  v = op(v, (uint32_t)__builtin_amdgcn_update_dpp((int)ident, (int)v, 0x141, 0xf, 0xf, false));  // row_half_mirror
  v = op(v, (uint32_t)__builtin_amdgcn_update_dpp((int)ident, (int)v, 0x140, 0xf, 0xf, false));  // row_mirror
  v = op(v, (uint32_t)__builtin_amdgcn_update_dpp((int)ident, (int)v, 0x142, 0xa, 0xf, false));  // row_bcast:15
  v = op(v, (uint32_t)__builtin_amdgcn_update_dpp((int)ident, (int)v, 0x143, 0xc, 0xf, false));  // row_bcast:31
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}
struct OpOr { __device__ uint32_t operator()(uint32_t a, uint32_t b) const { return a | b; } };
struct OpMin { __device__ uint32_t operator()(uint32_t a, uint32_t b) const { return a < b ? a : b; } };
struct OpMax { __device__ uint32_t operator()(uint32_t a, uint32_t b) const { return a > b ? a : b; } };
struct OpAdd { __device__ uint32_t operator()(uint32_t a, uint32_t b) const { return a + b; } };
__device__ inline uint32_t wave_or_dpp(uint32_t v) { return wave_reduce_dpp(v, OpOr(), 0u); }
// Exclusive prefix sum over the lanes of a wave through DPP: an inclusive
// scan within each 16-lane row (shifts by 1, 2, 4, 8; lanes shifted in from
// before the row read 0), then row 0's total into row 1 and row 2's into row
// 3 (broadcast of lane 15), then the first half's total into the second
// (broadcast of lane 31); no LDS round trip.
__device__ inline uint32_t wave_excl_sum_dpp(uint32_t v) {
  uint32_t x = v;
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);  // row_shr:1
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);  // row_shr:2
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);  // row_shr:4
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);  // row_shr:8
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);  // row_bcast:15
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return x - v;
}
__device__ inline uint32_t wave_min_dpp(uint32_t v) { return wave_reduce_dpp(v, OpMin(), 0xffffffffu); }
__device__ inline uint32_t wave_max_dpp(uint32_t v) { return wave_reduce_dpp(v, OpMax(), 0u); }
__device__ inline uint32_t wave_sum_dpp(uint32_t v) { return wave_reduce_dpp(v, OpAdd(), 0u); }

// Index of this wave in its workgroup, as a wave-uniform (scalar) value.
__device__ inline uint32_t wave_index() { return __builtin_amdgcn_readfirstlane(threadIdx.x / kWave); }

// number of set bits of m below this lane
__device__ inline uint32_t lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

}  // namespace chr
