// mc.hip -- marching cubes on gfx950 (Sec. I: isosurface generation;
// Sec. II.B: the per-cell case that topology preservation keeps).
//
// The field is reduced once to one bit per point (f < k) in 64-bit words
// along x; everything after that works on words:
//  1. k_mc_bits:  coalesced streaming pass, a ballot per 64 points.
//  2. k_mc_count: one lane per word: the word's crossing +x/+y/+z edges
//     (XORs of neighbouring words, popcount) and the triangles of the word's
//     active cells (cells whose 8 corners disagree, iterated as set bits;
//     triangle count from the generated table in LDS).
//  3. scan of the per-word {vertices, triangles}.
//  4. k_mc_emit:  one lane per word: vertices in (point, axis) order, then
//     triangles in (cell, table order) order; the id of the vertex on an edge
//     owned by point x' of word W is W's vertex base plus the popcount of W's
//     crossing masks below x' -- no per-point id array.
#include "chr_plan.h"
#include "mc_table.h"

namespace chr {
namespace {

constexpr int kBS = 256;
constexpr int kWaves = kBS / kWave;
constexpr int kWordsPerWave = 16;

constexpr mct::Table kTable = mct::make_table();
__constant__ mct::Table c_table = kTable;

typedef unsigned long long u64;

// f < k for 64 consecutive points per word; a wave covers kWordsPerWave
// words with all loads issued before the ballots.
__global__ __launch_bounds__(kBS) void k_mc_bits(McPlan M) {
  const int64_t nwords = M.nrows * M.nw;
  const int64_t w0 = ((int64_t)blockIdx.x * kWaves + threadIdx.x / kWave) * kWordsPerWave;
  if (w0 >= nwords) return;
  const int lane = lane_id();
  const int64_t nx = M.n[2];
  float v[kWordsPerWave];
#pragma unroll
  for (int k = 0; k < kWordsPerWave; k++) {
    const int64_t wi = w0 + k;
    v[k] = 0.f;
    if (wi < nwords) {
      const int64_t row = wi / M.nw, x = (wi - row * M.nw) * 64 + lane;
      if (x < nx) v[k] = M.f[row * nx + x];
    }
  }
#pragma unroll
  for (int k = 0; k < kWordsPerWave; k++) {
    const int64_t wi = w0 + k;
    bool below = false;
    if (wi < nwords) {
      const int64_t row = wi / M.nw, x = (wi - row * M.nw) * 64 + lane;
      below = (x < nx) && (v[k] < M.k);
    }
    const u64 m = __ballot(below);
    if (lane == 0 && wi < nwords) M.bits[wi] = m;
  }
}

struct WordCtx {
  int64_t row, w, z, y;
  u64 valid, validx;   // points of the word / points with a +x neighbour
};

__device__ inline WordCtx word_ctx(const McPlan &M, int64_t gw) {
  WordCtx c;
  c.row = gw / M.nw;
  c.w = gw - c.row * M.nw;
  c.z = c.row / M.n[1];
  c.y = c.row - c.z * M.n[1];
  const int64_t rem = M.n[2] - c.w * 64;
  c.valid = rem >= 64 ? ~0ull : ((1ull << rem) - 1ull);
  const int64_t remx = rem - 1;
  c.validx = remx >= 64 ? ~0ull : (remx <= 0 ? 0ull : ((1ull << remx) - 1ull));
  return c;
}

__device__ inline u64 bitsw(const McPlan &M, int64_t row, int64_t w) {
  return (w < M.nw) ? M.bits[row * M.nw + w] : 0ull;
}

struct Cross {
  u64 cx, cy, cz;
};

// Crossing masks of the owned +x/+y/+z edges of word w of point row (z, y).
__device__ inline Cross cross_of(const McPlan &M, int64_t z, int64_t y, int64_t w) {
  Cross c{0, 0, 0};
  if (w >= M.nw) return c;
  const int64_t row = z * M.n[1] + y;
  const int64_t rem = M.n[2] - w * 64;
  const u64 valid = rem >= 64 ? ~0ull : ((1ull << rem) - 1ull);
  const int64_t remx = rem - 1;
  const u64 validx = remx >= 64 ? ~0ull : (remx <= 0 ? 0ull : ((1ull << remx) - 1ull));
  const u64 m = bitsw(M, row, w);
  c.cx = (m ^ ((m >> 1) | (bitsw(M, row, w + 1) << 63))) & validx;
  if (y + 1 < M.n[1]) c.cy = (m ^ bitsw(M, row + 1, w)) & valid;
  if (z + 1 < M.n[0]) c.cz = (m ^ bitsw(M, row + M.n[1], w)) & valid;
  return c;
}

__device__ inline u64 shr1(u64 m, u64 next) { return (m >> 1) | (next << 63); }

// The 8 corner masks of the cells of word w of cell row `row`.
struct Corners {
  u64 m[8];
};

__device__ inline Corners corners_of(const McPlan &M, int64_t row, int64_t w) {
  Corners C;
  const int64_t r[4] = {row, row + 1, row + M.n[1], row + M.n[1] + 1};  // (dy,dz) = 00, 10, 01, 11
  for (int i = 0; i < 4; i++) {
    const u64 a = bitsw(M, r[i], w), b = bitsw(M, r[i], w + 1);
    C.m[2 * i] = a;               // corner dx = 0
    C.m[2 * i + 1] = shr1(a, b);  // corner dx = 1
  }
  return C;
}

__device__ inline uint32_t case_at(const Corners &C, int i) {
  uint32_t cs = 0;
#pragma unroll
  for (int v = 0; v < 8; v++) cs |= (uint32_t)((C.m[v] >> i) & 1ull) << v;
  return cs;
}

__device__ inline u64 active_cells(const Corners &C, u64 validx) {
  u64 any = 0, all = ~0ull;
#pragma unroll
  for (int v = 0; v < 8; v++) { any |= C.m[v]; all &= C.m[v]; }
  return any & ~all & validx;
}

__global__ __launch_bounds__(kBS) void k_mc_count(McPlan M) {
  __shared__ uint8_t ntri[256];
  for (int i = threadIdx.x; i < 256; i += kBS) ntri[i] = c_table.ntri[i];
  __syncthreads();
  const int64_t gw = (int64_t)blockIdx.x * kBS + threadIdx.x;
  if (gw >= M.nrows * M.nw) return;
  const WordCtx c = word_ctx(M, gw);
  const Cross x = cross_of(M, c.z, c.y, c.w);
  const uint32_t nv = (uint32_t)(__popcll(x.cx) + __popcll(x.cy) + __popcll(x.cz));
  uint32_t nt = 0;
  if (c.y + 1 < M.n[1] && c.z + 1 < M.n[0]) {
    const Corners C = corners_of(M, c.row, c.w);
    u64 act = active_cells(C, c.validx);
    while (act) {
      const int i = __ffsll((long long)act) - 1;
      act &= act - 1;
      nt += ntri[case_at(C, i)];
    }
  }
  M.cnt[gw] = U4{nv, nt, 0u, 0u};
}

__device__ inline float interp(float fa, float fb, float k) {
  return __fdiv_rn(__fsub_rn(k, fa), __fsub_rn(fb, fa));
}

// Vertex-id context of one owner row for word w: crossing masks of words w
// and w+1 and their vertex bases.
struct Owner {
  Cross c0, c1;
  uint64_t v0, v1;
};

__device__ inline int popc3_below(const Cross &c, int x) {
  const u64 bm = (x >= 64) ? ~0ull : ((1ull << x) - 1ull);
  return __popcll(c.cx & bm) + __popcll(c.cy & bm) + __popcll(c.cz & bm);
}

__global__ __launch_bounds__(kBS) void k_mc_emit(McPlan M) {
  __shared__ mct::Table tab;
  {
    const uint8_t *src = reinterpret_cast<const uint8_t *>(&c_table);
    uint8_t *dst = reinterpret_cast<uint8_t *>(&tab);
    for (int i = threadIdx.x; i < (int)sizeof(mct::Table); i += kBS) dst[i] = src[i];
  }
  __syncthreads();
  const int64_t gw = (int64_t)blockIdx.x * kBS + threadIdx.x;
  if (gw >= M.nrows * M.nw) return;
  const U4 p0 = M.P[gw], p1 = M.P[gw + 1];
  if (p0.x == p1.x && p0.y == p1.y) return;
  const WordCtx c = word_ctx(M, gw);
  const int64_t n1 = M.n[1], n2 = M.n[2];
  const float *f = M.f;
  const float k = M.k, sp = M.spacing;

  // vertices of this word's points, in (point, axis) order
  if (p1.x != p0.x) {
    const Cross x = cross_of(M, c.z, c.y, c.w);
    uint64_t id = p0.x;
    u64 pts = x.cx | x.cy | x.cz;
    const float py = (float)c.y, pz = (float)c.z;
    while (pts) {
      const int i = __ffsll((long long)pts) - 1;
      pts &= pts - 1;
      const int64_t xx = c.w * 64 + i;
      const size_t gi = ((size_t)c.z * n1 + c.y) * n2 + xx;
      const float fa = f[gi];
      const float px = (float)xx;
      if ((x.cx >> i) & 1ull) {
        if ((int64_t)id < M.cap_v) {
          const float t = interp(fa, f[gi + 1], k);
          float *v = M.verts + 3 * id;
          v[0] = __fmul_rn(__fadd_rn(px, t), sp); v[1] = __fmul_rn(py, sp); v[2] = __fmul_rn(pz, sp);
        }
        id++;
      }
      if ((x.cy >> i) & 1ull) {
        if ((int64_t)id < M.cap_v) {
          const float t = interp(fa, f[gi + n2], k);
          float *v = M.verts + 3 * id;
          v[0] = __fmul_rn(px, sp); v[1] = __fmul_rn(__fadd_rn(py, t), sp); v[2] = __fmul_rn(pz, sp);
        }
        id++;
      }
      if ((x.cz >> i) & 1ull) {
        if ((int64_t)id < M.cap_v) {
          const float t = interp(fa, f[gi + (size_t)n1 * n2], k);
          float *v = M.verts + 3 * id;
          v[0] = __fmul_rn(px, sp); v[1] = __fmul_rn(py, sp); v[2] = __fmul_rn(__fadd_rn(pz, t), sp);
        }
        id++;
      }
    }
  }

  // triangles of this word's cells, in (cell, table order) order
  if (p1.y != p0.y) {
    const int64_t rows[4] = {c.row, c.row + 1, c.row + n1, c.row + n1 + 1};
    const int64_t ry[4] = {c.y, c.y + 1, c.y, c.y + 1}, rz[4] = {c.z, c.z, c.z + 1, c.z + 1};
    Owner own[4];
    for (int r = 0; r < 4; r++) {
      own[r].c0 = cross_of(M, rz[r], ry[r], c.w);
      own[r].c1 = cross_of(M, rz[r], ry[r], c.w + 1);
      own[r].v0 = M.P[rows[r] * M.nw + c.w].x;
      own[r].v1 = (c.w + 1 < M.nw) ? M.P[rows[r] * M.nw + c.w + 1].x : 0;
    }
    const Corners C = corners_of(M, c.row, c.w);
    u64 act = active_cells(C, c.validx);
    uint64_t tid = p0.y;
    while (act) {
      const int i = __ffsll((long long)act) - 1;
      act &= act - 1;
      const uint32_t cs = case_at(C, i);
      const int nt = tab.ntri[cs];
      for (int t = 0; t < nt; t++, tid++) {
        int32_t ids[3];
        for (int q = 0; q < 3; q++) {
          const int e = tab.tri[cs][3 * t + q];
          const int axis = e >> 2, i2 = e & 3;
          int dx = 0, dy = 0, dz = 0;
          if (axis == 0) { dy = i2 & 1; dz = i2 >> 1; }
          if (axis == 1) { dx = i2 & 1; dz = i2 >> 1; }
          if (axis == 2) { dx = i2 & 1; dy = i2 >> 1; }
          const Owner &o = own[dy + 2 * dz];
          const int xo = i + dx;
          uint64_t id;
          u64 mx, my;
          int bit;
          if (xo < 64) { id = o.v0 + popc3_below(o.c0, xo); mx = o.c0.cx; my = o.c0.cy; bit = xo; }
          else { id = o.v1; mx = o.c1.cx; my = o.c1.cy; bit = 0; }
          if (axis >= 1) id += (mx >> bit) & 1ull;
          if (axis >= 2) id += (my >> bit) & 1ull;
          ids[q] = (int32_t)id;
        }
        if ((int64_t)tid < M.cap_t) {
          int32_t *o = M.tris + 3 * tid;
          o[0] = ids[0]; o[1] = ids[1]; o[2] = ids[2];
        }
      }
    }
  }
}

__global__ void k_mc_counts(McPlan M) {
  if (threadIdx.x == 0) {
    const int64_t n = M.nrows * M.nw;
    M.counts[0] = (int64_t)M.P[n].x;
    M.counts[1] = (int64_t)M.P[n].y;
  }
}

// Case of every cell (one lane per word of cells).
__global__ __launch_bounds__(kBS) void k_mc_cases(McPlan M) {
  const int64_t gw = (int64_t)blockIdx.x * kBS + threadIdx.x;
  if (gw >= M.nrows * M.nw) return;
  const WordCtx c = word_ctx(M, gw);
  if (c.y + 1 >= M.n[1] || c.z + 1 >= M.n[0]) return;
  const int64_t cy = M.n[1] - 1, cx = M.n[2] - 1;
  const Corners C = corners_of(M, c.row, c.w);
  for (int i = 0; i < 64; i++) {
    const int64_t x = c.w * 64 + i;
    if (x >= cx) break;
    M.cases[(c.z * cy + c.y) * cx + x] = (uint8_t)case_at(C, i);
  }
}

__global__ __launch_bounds__(kBS) void k_range(const float *__restrict__ f, int64_t n, uint32_t *acc) {
  uint32_t mn = 0xffffffffu, mx = 0u, nf = 0u;
  for (int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBS) {
    const float v = f[i];
    if (!isfinite(v)) { nf++; continue; }
    const uint32_t o = ord_of(v);
    mn = min(mn, o);
    mx = max(mx, o);
  }
  mn = wave_min_u(mn);
  mx = wave_max_u(mx);
  nf = wave_sum_u(nf);
  if (lane_id() == 0) {
    atomicMin(&acc[0], mn);
    atomicMax(&acc[1], mx);
    if (nf) atomicAdd(&acc[2], nf);
  }
}

__global__ void k_range_init(uint32_t *acc) {
  if (threadIdx.x == 0) { acc[0] = 0xffffffffu; acc[1] = 0u; acc[2] = 0u; acc[3] = 0u; }
}

__global__ void k_range_fin(uint32_t *acc) {
  if (threadIdx.x == 0) {
    const float mn = of_ord(acc[0]), mx = of_ord(acc[1]);
    acc[0] = __float_as_uint(mn);
    acc[1] = __float_as_uint(mx);
  }
}

}  // namespace

void launch_mc(const McPlan &p, U4 *scan_tmp, hipStream_t s) {
  const int64_t nwords = p.nrows * p.nw;
  prof_mark("k_mc_bits", s, 0);
  k_mc_bits<<<dim3((unsigned)ceil_div(nwords, (int64_t)kWaves * kWordsPerWave)), dim3(kBS), 0, s>>>(p);
  prof_mark("k_mc_bits", s, 1);
  prof_mark("k_mc_count", s, 0);
  k_mc_count<<<dim3((unsigned)ceil_div(nwords, kBS)), dim3(kBS), 0, s>>>(p);
  prof_mark("k_mc_count", s, 1);
  scan_u4(p.cnt, p.P, nwords, scan_tmp, s);
  prof_mark("k_mc_emit", s, 0);
  k_mc_emit<<<dim3((unsigned)ceil_div(nwords, kBS)), dim3(kBS), 0, s>>>(p);
  prof_mark("k_mc_emit", s, 1);
  k_mc_counts<<<dim3(1), dim3(64), 0, s>>>(p);
}

void launch_mc_cases(const McPlan &p, hipStream_t s) {
  const int64_t nwords = p.nrows * p.nw;
  k_mc_bits<<<dim3((unsigned)ceil_div(nwords, (int64_t)kWaves * kWordsPerWave)), dim3(kBS), 0, s>>>(p);
  if (p.n[0] > 1 && p.n[1] > 1 && p.n[2] > 1)
    k_mc_cases<<<dim3((unsigned)ceil_div(nwords, kBS)), dim3(kBS), 0, s>>>(p);
}

void launch_range(const float *f, int64_t n, float *out, hipStream_t s) {
  uint32_t *acc = reinterpret_cast<uint32_t *>(out);
  k_range_init<<<1, 64, 0, s>>>(acc);
  int64_t blocks = ceil_div(n, kBS * 8);
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  k_range<<<dim3((unsigned)blocks), dim3(kBS), 0, s>>>(f, n, acc);
  k_range_fin<<<1, 64, 0, s>>>(acc);
}

void mc_table_host(uint8_t *ntri, int8_t *tri) {
  for (int c = 0; c < 256; c++) {
    ntri[c] = kTable.ntri[c];
    for (int i = 0; i < 15; i++) tri[15 * c + i] = kTable.tri[c][i];
  }
}

}  // namespace chr
