// mc.hip -- marching cubes on gfx950 (Sec. I: isosurface generation;
// Sec. II.B: the per-cell case that topology preservation keeps).
//
// The field is reduced once to one bit per point (f < k) in 64-bit words
// along x; everything after that works on words:
//  1. k_mc_bits:   coalesced streaming pass, a ballot per 64 points.
//  2. k_mc_count:  one lane per word: its crossing +x/+y/+z edges (XORs of
//     neighbouring words, popcount), the points carrying them, its active
//     cells (corners disagree) and their triangles, counted on the 64 cells
//     at once from the crossed cell edges (E - 2 per single-loop cell, table
//     corrections for the rare cells that may hold several loops).
//  3. scan of the per-word {vertices, triangles, crossing points, active cells}.
//  4. k_mc_expand: compact lists of the crossing points and of the active
//     cells, written word after word by the lanes of the word's set bits
//     (consecutive entries, coalesced stores).
//  5. k_mc_verts / k_mc_tris: one lane per list entry, so lanes stay dense
//     however sparse the surface is.  The id of the vertex on an edge owned by
//     point x' of word W is W's vertex base plus the popcount of W's crossing
//     masks below x' -- no per-point id array.  A workgroup of k_mc_tris
//     takes 256 consecutive active cells: its first triangle id from the
//     word prefix and the cells before it in their word, the others by a
//     workgroup scan of the cells' triangle counts.
#include "chr_plan.h"
#include "mc_table.h"

namespace chr {
namespace {

constexpr int kBS = 256;
constexpr int kWaves = kBS / kWave;
constexpr int kWordsPerWave = 8;

constexpr mct::Table kTable = mct::make_table();
__constant__ mct::Table c_table = kTable;
static_assert(mct::loop_rule_holds(kTable), "a case outside multi_loop_possible has more than one loop");
constexpr mct::LoopFix kFix = mct::make_loop_fix(kTable);
__constant__ mct::LoopFix c_fix = kFix;

constexpr int max_ntri(const mct::Table &t) {
  int m = 0;
  for (int c = 0; c < 256; c++) m = t.ntri[c] > m ? t.ntri[c] : m;
  return m;
}
constexpr int kMaxTri = max_ntri(kTable);  // triangles of one cell at most
static_assert(kMaxTri <= 5, "triangle staging assumes at most 5 triangles per cell");

typedef unsigned long long u64;

// f < k for 64 consecutive points per word.  One wave per row of points;
// it issues the loads of kWordsPerWave words (unconditional: past the row's
// end a lane reads the row's last point and is masked) before their ballots,
// and lane j stores word j, so the words of a step take one store.
__global__ __launch_bounds__(kBS) void k_mc_bits(McPlan M) {
  const int64_t row = (int64_t)blockIdx.x * kWaves + wave_index();
  if (row >= M.nrows) return;
  const int lane = lane_id();
  const uint32_t nx = (uint32_t)M.n[2], nw = (uint32_t)M.nw;
  const uint32_t rz = fdiv((uint32_t)row, M.d_n1), ry = (uint32_t)row - rz * (uint32_t)M.n[1];
  const char *__restrict__ fb = reinterpret_cast<const char *>(M.f + (int64_t)rz * M.pz + (int64_t)ry * M.py);
  u64 *out = M.bits + row * M.nw;
  const float k = M.k;
  for (uint32_t w0 = 0; w0 < nw; w0 += kWordsPerWave) {
    float v[kWordsPerWave];
#pragma unroll
    for (int j = 0; j < kWordsPerWave; j++) {
      const uint32_t x = (w0 + j) * 64u + (uint32_t)lane;
      v[j] = ldf(fb, min(x, nx - 1u) * 4u);
    }
    u64 mine = 0;
#pragma unroll
    for (int j = 0; j < kWordsPerWave; j++) {
      const uint32_t x = (w0 + j) * 64u + (uint32_t)lane;
      const u64 m = __ballot((x < nx) && (v[j] < k));
      if (lane == j) mine = m;
    }
    if (lane < kWordsPerWave && w0 + (uint32_t)lane < nw) out[w0 + lane] = mine;
  }
}

struct WordCtx {
  int64_t row, w, z, y;
  u64 valid, validx;   // points of the word / points with a +x neighbour
};

// Word indices are below 2^26 (the launcher keeps padded points below
// 2^32), so the split uses the launcher's 32-bit divisors.
__device__ inline WordCtx word_ctx(const McPlan &M, int64_t gw64) {
  WordCtx c;
  const uint32_t gw = (uint32_t)gw64;
  const uint32_t row = fdiv(gw, M.d_nw), z = fdiv(row, M.d_n1);
  c.row = row;
  c.w = gw - row * (uint32_t)M.nw;
  c.z = z;
  c.y = row - z * (uint32_t)M.n[1];
  const int32_t rem = (int32_t)M.n[2] - (int32_t)c.w * 64;
  c.valid = rem >= 64 ? ~0ull : ((1ull << rem) - 1ull);
  const int32_t remx = rem - 1;
  c.validx = remx >= 64 ? ~0ull : (remx <= 0 ? 0ull : ((1ull << remx) - 1ull));
  return c;
}

// 32-bit form (word indices are below 2^26: padded points are below 2^32).
struct WordCtx32 {
  uint32_t row, w, z, y;
};

__device__ inline WordCtx32 word_ctx32(const McPlan &M, uint32_t gw) {
  WordCtx32 c;
  c.row = fdiv(gw, M.d_nw);
  c.w = gw - c.row * (uint32_t)M.nw;
  c.z = fdiv(c.row, M.d_n1);
  c.y = c.row - c.z * (uint32_t)M.n[1];
  return c;
}

// Word w of point row `row`, 0 past the row's last word.  The load itself is
// unconditional (clamped to the last word), so that the loads of a lane's
// words can all be in flight together.
__device__ inline u64 bitsw(const McPlan &M, uint32_t row, uint32_t w) {
  const uint32_t nw = (uint32_t)M.nw;
  const bool in = w < nw;
  const u64 v = M.bits[row * nw + (in ? w : nw - 1)];
  return in ? v : 0ull;
}

struct Cross {
  u64 cx, cy, cz;
};

// Crossing masks of the owned +x/+y/+z edges of word w of point row (z, y)
// (all zero for a word past the row's end).  Rows past the grid are read as
// the row itself and masked off.
__device__ inline Cross cross_of(const McPlan &M, uint32_t z, uint32_t y, uint32_t w) {
  const uint32_t nw = (uint32_t)M.nw, n1 = (uint32_t)M.n[1];
  const bool inw = w < nw;
  const uint32_t wc = inw ? w : nw - 1;
  const uint32_t row = z * n1 + y;
  const int32_t rem = (int32_t)M.n[2] - (int32_t)wc * 64;
  const u64 valid = rem >= 64 ? ~0ull : ((1ull << rem) - 1ull);
  const int32_t remx = rem - 1;
  const u64 validx = remx >= 64 ? ~0ull : (remx <= 0 ? 0ull : ((1ull << remx) - 1ull));
  const bool hy = y + 1 < n1, hz = z + 1 < (uint32_t)M.n[0];
  const u64 m = bitsw(M, row, wc);
  const u64 mn = bitsw(M, row, wc + 1);
  const u64 my = bitsw(M, hy ? row + 1 : row, wc);
  const u64 mz = bitsw(M, hz ? row + n1 : row, wc);
  Cross c;
  c.cx = inw ? (m ^ ((m >> 1) | (mn << 63))) & validx : 0ull;
  c.cy = (inw && hy) ? (m ^ my) & valid : 0ull;
  c.cz = (inw && hz) ? (m ^ mz) & valid : 0ull;
  return c;
}

__device__ inline u64 shr1(u64 m, u64 next) { return (m >> 1) | (next << 63); }

// The 8 corner masks of the cells of word w of cell row `row`.
struct Corners {
  u64 m[8];
};

__device__ inline Corners corners_of(const McPlan &M, uint32_t row, uint32_t w) {
  Corners C;
  const uint32_t n1 = (uint32_t)M.n[1];
  const uint32_t r[4] = {row, row + 1, row + n1, row + n1 + 1};  // (dy,dz) = 00, 10, 01, 11
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

// Triangles of the active cells `act` of a word with corner masks C: the
// crossed cell edges, minus two per active cell, plus the table's correction
// of each cell whose case may hold several loops (any ambiguous face, or the
// below or the above corners a lone body-diagonal pair; few cells).
__device__ inline uint32_t word_tris(const Corners &C, u64 act, const int8_t *fix) {
  uint32_t e = 0;
#pragma unroll
  for (int k = 0; k < 12; k++) {
    const mct::Edge E = mct::edge_of(k);
    e += (uint32_t)__popcll((C.m[E.lo] ^ C.m[E.hi]) & act);
  }
  u64 multi = 0;
#pragma unroll
  for (int f = 0; f < 6; f++) {
    const u64 a = C.m[mct::kFaces[f][0]], b = C.m[mct::kFaces[f][1]];
    const u64 c = C.m[mct::kFaces[f][2]], d = C.m[mct::kFaces[f][3]];
    multi |= ~(a ^ c) & ~(b ^ d) & (a ^ b);
  }
  u64 por[4], pand[4];
#pragma unroll
  for (int p = 0; p < 4; p++) {
    por[p] = C.m[mct::kBodyDiag[p][0]] | C.m[mct::kBodyDiag[p][1]];
    pand[p] = C.m[mct::kBodyDiag[p][0]] & C.m[mct::kBodyDiag[p][1]];
  }
  const u64 o01 = por[0] | por[1], o23 = por[2] | por[3];
  const u64 a01 = pand[0] & pand[1], a23 = pand[2] & pand[3];
  const u64 orest[4] = {por[1] | o23, por[0] | o23, o01 | por[3], o01 | por[2]};
  const u64 arest[4] = {pand[1] & a23, pand[0] & a23, a01 & pand[3], a01 & pand[2]};
#pragma unroll
  for (int p = 0; p < 4; p++) multi |= (pand[p] & ~orest[p]) | (~por[p] & arest[p]);
  multi &= act;
  int t = (int)e - 2 * __popcll(act);
  while (multi) {
    const int i = __ffsll((long long)multi) - 1;
    multi &= multi - 1;
    t += fix[case_at(C, i)];
  }
  return (uint32_t)t;
}

__global__ __launch_bounds__(kBS) void k_mc_count(McPlan M) {
  __shared__ int8_t fix[256];
  for (int i = threadIdx.x; i < 256; i += kBS) fix[i] = c_fix.d[i];
  __syncthreads();
  const int64_t gw = (int64_t)blockIdx.x * kBS + threadIdx.x;
  if (gw >= M.nrows * M.nw) return;
  const WordCtx c = word_ctx(M, gw);
  const Cross x = cross_of(M, c.z, c.y, c.w);
  const uint32_t nv = (uint32_t)(__popcll(x.cx) + __popcll(x.cy) + __popcll(x.cz));
  const uint32_t npv = (uint32_t)__popcll(x.cx | x.cy | x.cz);
  uint32_t nt = 0, nac = 0;
  if (c.y + 1 < M.n[1] && c.z + 1 < M.n[0]) {
    const Corners C = corners_of(M, c.row, c.w);
    const u64 act = active_cells(C, c.validx);
    nac = (uint32_t)__popcll(act);
    if (act) nt = word_tris(C, act, fix);
  }
  M.cnt[gw] = nv | (nt << 8) | (npv << 17) | (nac << 24);   // the packed record scan_u4_packed reads
}

__device__ inline float interp(float fa, float fb, float k) {
  return __fdiv_rn(__fsub_rn(k, fa), __fsub_rn(fb, fa));
}

__device__ inline int popc3_below(const Cross &c, int x) {
  const u64 bm = (x >= 64) ? ~0ull : ((1ull << x) - 1ull);
  return __popcll(c.cx & bm) + __popcll(c.cy & bm) + __popcll(c.cz & bm);
}

// Lists the crossing points and the active cells of the wave's 64 words
// (entries word*64 + bit; a word's entries are written only if the whole
// list up to it fits: lists are whole or unused).  Two ways: each lane walks
// its own word's bits (as many steps as the fullest word, one scattered
// store per step), or word after word the lanes of the word's set bits
// write its entries at consecutive positions (one step per word with
// entries, every store coalesced).  A wave takes the second where its
// fullest words have more bits than it has words with entries (a dense
// surface).
__global__ __launch_bounds__(kBS) void k_mc_expand(McPlan M) {
  const uint32_t nwords = (uint32_t)(M.nrows * M.nw);
  const uint32_t gw0 = blockIdx.x * kBS + wave_index() * kWave;   // the wave's first word
  const int lane = lane_id();
  const uint32_t gw = gw0 + (uint32_t)lane;
  u64 pts = 0, act = 0;
  uint32_t bz = 0, bw = 0;
  if (gw < nwords) {
    const U4 p0 = M.P[gw], p1 = M.P[gw + 1];
    bz = p0.z;
    bw = p0.w;
    const bool okz = p1.z != p0.z && (int64_t)p1.z <= M.cap_pv;
    const bool okw = p1.w != p0.w && (int64_t)p1.w <= M.cap_ac;
    if (okz || okw) {
      const WordCtx c = word_ctx(M, gw);
      if (okz) {
        const Cross x = cross_of(M, c.z, c.y, c.w);
        pts = x.cx | x.cy | x.cz;
      }
      if (okw) act = active_cells(corners_of(M, c.row, c.w), c.validx);
    }
  }
  u64 todo = __ballot(pts != 0ull || act != 0ull);
  const uint32_t steps = wave_max_dpp((uint32_t)__popcll(pts)) + wave_max_dpp((uint32_t)__popcll(act));
  if (steps < (uint32_t)__popcll(todo)) {
    uint32_t r = bz;
    while (pts) {
      const int i = __ffsll((long long)pts) - 1;
      pts &= pts - 1;
      M.vlist[r++] = gw * 64u + (uint32_t)i;
    }
    r = bw;
    while (act) {
      const int i = __ffsll((long long)act) - 1;
      act &= act - 1;
      M.clist[r++] = gw * 64u + (uint32_t)i;
    }
    return;
  }
  while (todo) {
    const int k = __ffsll((long long)todo) - 1;
    todo &= todo - 1;
    const u64 pk = ((u64)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(pts >> 32), k) << 32) |
                   (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)pts, k);
    const u64 ak = ((u64)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(act >> 32), k) << 32) |
                   (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)act, k);
    const uint32_t code = (gw0 + (uint32_t)k) * 64u + (uint32_t)lane;
    if (__builtin_amdgcn_inverse_ballot_w64(pk))
      M.vlist[(uint32_t)__builtin_amdgcn_readlane((int)bz, k) + lanes_below(pk)] = code;
    if (__builtin_amdgcn_inverse_ballot_w64(ak))
      M.clist[(uint32_t)__builtin_amdgcn_readlane((int)bw, k) + lanes_below(ak)] = code;
  }
}

// First triangle id of every 256th active cell, where a k_mc_tris
// workgroup's range starts: the triangle prefix of the cell's word plus the
// triangles of the word's active cells before it (one wave per such cell,
// one lane per cell of its word; run by the waves of k_mc_verts before
// their vertices).
__device__ inline void tile_bases(const McPlan &M, const uint8_t *ntri) {
  const uint32_t nwords = (uint32_t)(M.nrows * M.nw);
  const uint32_t n = (int64_t)M.P[nwords].w <= M.cap_ac ? M.P[nwords].w : 0u;
  const uint32_t ntiles = (n + kBS - 1) / kBS;
  const int lane = lane_id();
  for (uint32_t t = blockIdx.x * kWaves + wave_index(); t < ntiles; t += gridDim.x * kWaves) {
    const uint32_t ent = M.clist[t * kBS];
    const WordCtx c = word_ctx(M, ent >> 6);
    const Corners C = corners_of(M, (uint32_t)c.row, (uint32_t)c.w);
    const u64 act = active_cells(C, c.validx);
    const uint32_t mine = ((act >> lane) & 1ull) && (uint32_t)lane < (ent & 63u) ? (uint32_t)ntri[case_at(C, lane)] : 0u;
    const uint32_t before = wave_sum_dpp(mine);
    if (lane == 0) M.tb[t] = M.P[ent >> 6].y + before;
  }
}

// One lane per crossing point: its vertices in axis order x, y, z (a lane's
// vertices are consecutive, and so are consecutive lanes').
__global__ __launch_bounds__(kBS) void k_mc_verts(McPlan M) {
  __shared__ uint8_t ntri[256];
  for (int i = threadIdx.x; i < 256; i += kBS) ntri[i] = c_table.ntri[i];
  __syncthreads();
  tile_bases(M, ntri);
  const uint32_t nwords = (uint32_t)(M.nrows * M.nw);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    // the mesh sizes (required sizes, also when they exceed the capacities)
    M.counts[0] = (int64_t)M.P[nwords].x;
    M.counts[1] = (int64_t)M.P[nwords].y;
  }
  const uint32_t n = (int64_t)M.P[nwords].z <= M.cap_pv ? M.P[nwords].z : 0u;  // lists are whole or unused
  const uint32_t n1 = (uint32_t)M.n[1], n2 = (uint32_t)M.n[2];
  const float *f = M.f;
  const float k = M.k, sp = M.spacing;
  for (uint32_t e = blockIdx.x * kBS + threadIdx.x; e < n; e += gridDim.x * kBS) {
    const uint32_t code = M.vlist[e];
    const uint32_t gw = code >> 6;
    const int i = code & 63;
    const WordCtx32 c = word_ctx32(M, gw);
    const Cross x = cross_of(M, c.z, c.y, c.w);
    uint64_t id = M.P[gw].x + (uint32_t)popc3_below(x, i);
    const uint32_t xx = c.w * 64u + (uint32_t)i;
    const size_t gi = (size_t)c.z * (size_t)M.pz + (size_t)c.y * (size_t)M.py + xx;
    // the point and its three neighbours, loaded together with the masks
    // (a missing neighbour reads the point itself and is never used)
    const float fa = f[gi];
    const float fx = f[xx + 1 < n2 ? gi + 1 : gi];
    const float fy = f[c.y + 1 < n1 ? gi + (size_t)M.py : gi];
    const float fz = f[c.z + 1 < (uint32_t)M.n[0] ? gi + (size_t)M.pz : gi];
    const float px = (float)(xx + M.org[2]), py = (float)(c.y + M.org[1]), pz = (float)(c.z + M.org[0]);
    if ((x.cx >> i) & 1ull) {
      if ((int64_t)id < M.cap_v) {
        const float t = interp(fa, fx, k);
        float *v = M.verts + 3 * id;
        v[0] = __fmul_rn(__fadd_rn(px, t), sp); v[1] = __fmul_rn(py, sp); v[2] = __fmul_rn(pz, sp);
      }
      id++;
    }
    if ((x.cy >> i) & 1ull) {
      if ((int64_t)id < M.cap_v) {
        const float t = interp(fa, fy, k);
        float *v = M.verts + 3 * id;
        v[0] = __fmul_rn(px, sp); v[1] = __fmul_rn(__fadd_rn(py, t), sp); v[2] = __fmul_rn(pz, sp);
      }
      id++;
    }
    if ((x.cz >> i) & 1ull) {
      if ((int64_t)id < M.cap_v) {
        const float t = interp(fa, fz, k);
        float *v = M.verts + 3 * id;
        v[0] = __fmul_rn(px, sp); v[1] = __fmul_rn(py, sp); v[2] = __fmul_rn(__fadd_rn(pz, t), sp);
      }
    }
  }
}

// Vertex id of an edge's owner point and that point's +x / +y crossing bits
// (the vertex on its +y edge follows the one on +x, the one on +z follows
// both).
struct Owner {
  uint32_t base, bx, by;
};

// One lane per active cell: the ids of its 12 edge vertices go to LDS, then
// its triangles in table order.  A workgroup takes 256 consecutive active
// cells, whose triangles are one contiguous id range starting at the id
// k_mc_verts found; a cell's offset in the range is a workgroup scan of
// the cells' triangle counts (at most 5: three ballots per wave).  The
// triangles are staged in LDS and written out coalesced.
__global__ __launch_bounds__(kBS) void k_mc_tris(McPlan M) {
  constexpr int kIdStride = 13;  // 12 edge ids per lane, odd stride against bank conflicts
  __shared__ mct::Table tab;
  __shared__ int32_t st[kBS * kMaxTri * 3];
  __shared__ int32_t sid[kBS * kIdStride];
  __shared__ uint32_t wsum[kWaves];
  {
    const uint8_t *src = reinterpret_cast<const uint8_t *>(&c_table);
    uint8_t *dst = reinterpret_cast<uint8_t *>(&tab);
    for (int i = threadIdx.x; i < (int)sizeof(mct::Table); i += kBS) dst[i] = src[i];
  }
  __syncthreads();
  const uint32_t nwords = (uint32_t)(M.nrows * M.nw);
  const uint32_t n = (int64_t)M.P[nwords].w <= M.cap_ac ? M.P[nwords].w : 0u;
  const uint32_t n1 = (uint32_t)M.n[1], nw = (uint32_t)M.nw;
  const uint32_t wave = wave_index();
  const int lane = lane_id();
  int32_t *my = sid + threadIdx.x * kIdStride;
  for (uint32_t e0 = blockIdx.x * kBS; e0 < n; e0 += gridDim.x * kBS) {
    const uint32_t e = e0 + threadIdx.x;
    const uint32_t tbase = M.tb[e0 / kBS];
    uint32_t nt = 0, cs = 0;
    if (e < n) {
      const uint32_t code = M.clist[e];
      const uint32_t gw = code >> 6;
      const int i = code & 63;
      const WordCtx32 c = word_ctx32(M, gw);
      // Every word this cell needs, loaded at once: point rows (z+dz, y+dy)
      // for dz, dy in 0..2 (not both 2), words w and w+1.  Rows and words
      // past the grid are read clamped and masked off below.
      const uint32_t n0 = (uint32_t)M.n[0], n2 = (uint32_t)M.n[2];
      const bool hy2 = c.y + 2 < n1, hz2 = c.z + 2 < n0, hn = c.w + 1 < nw;
      const uint32_t wn = hn ? c.w + 1 : c.w;
      const uint32_t ra0 = c.row, ra1 = ra0 + 1, ra2 = hy2 ? ra0 + 2 : ra1;
      const uint32_t rb0 = ra0 + n1, rb1 = rb0 + 1, rb2 = hy2 ? rb0 + 2 : rb1;
      const uint32_t rc0 = hz2 ? rb0 + n1 : rb0, rc1 = hz2 ? rb1 + n1 : rb1;
      const u64 *__restrict__ B = M.bits;
      const u64 a0 = B[ra0 * nw + c.w], a0n = B[ra0 * nw + wn], a1 = B[ra1 * nw + c.w], a1n = B[ra1 * nw + wn];
      const u64 a2 = B[ra2 * nw + c.w], a2n = B[ra2 * nw + wn];
      const u64 b0 = B[rb0 * nw + c.w], b0n = B[rb0 * nw + wn], b1 = B[rb1 * nw + c.w], b1n = B[rb1 * nw + wn];
      const u64 b2 = B[rb2 * nw + c.w];
      const u64 c0 = B[rc0 * nw + c.w], c1 = B[rc1 * nw + c.w];
      const uint32_t v0 = M.P[ra0 * nw + c.w].x, v1 = M.P[ra1 * nw + c.w].x;
      const uint32_t v2 = M.P[rb0 * nw + c.w].x, v3 = M.P[rb1 * nw + c.w].x;
      const uint32_t v0n = M.P[ra0 * nw + wn].x, v1n = M.P[ra1 * nw + wn].x, v2n = M.P[rb0 * nw + wn].x;
      // corners of the cells of word w (rows (dy,dz) = 00, 10, 01, 11)
      const u64 nx0 = hn ? a0n : 0ull, nx1 = hn ? a1n : 0ull, nx2 = hn ? b0n : 0ull, nx3 = hn ? b1n : 0ull;
      Corners C;
      C.m[0] = a0; C.m[1] = shr1(a0, nx0);
      C.m[2] = a1; C.m[3] = shr1(a1, nx1);
      C.m[4] = b0; C.m[5] = shr1(b0, nx2);
      C.m[6] = b1; C.m[7] = shr1(b1, nx3);
      cs = case_at(C, i);
      nt = tab.ntri[cs];
      // crossing masks of the four owner rows at word w
      const int64_t rem = (int64_t)n2 - (int64_t)c.w * 64;
      const u64 valid = rem >= 64 ? ~0ull : ((1ull << rem) - 1ull);
      const u64 validx = rem - 1 >= 64 ? ~0ull : (rem - 1 <= 0 ? 0ull : ((1ull << (rem - 1)) - 1ull));
      Cross k0, k1, k2, k3;
      k0.cx = (a0 ^ shr1(a0, nx0)) & validx; k0.cy = (a0 ^ a1) & valid; k0.cz = (a0 ^ b0) & valid;
      k1.cx = (a1 ^ shr1(a1, nx1)) & validx; k1.cy = hy2 ? (a1 ^ a2) & valid : 0ull; k1.cz = (a1 ^ b1) & valid;
      k2.cx = (b0 ^ shr1(b0, nx2)) & validx; k2.cy = (b0 ^ b1) & valid; k2.cz = hz2 ? (b0 ^ c0) & valid : 0ull;
      k3.cx = (b1 ^ shr1(b1, nx3)) & validx; k3.cy = hy2 ? (b1 ^ b2) & valid : 0ull; k3.cz = hz2 ? (b1 ^ c1) & valid : 0ull;
      // the first point of word w+1 (owner of the +x corner when i = 63):
      // its +x / +y crossing bits
      const bool x1 = (uint64_t)(c.w + 1) * 64u + 1u < n2;  // it has a +x neighbour
      const uint32_t a0x = x1 ? (uint32_t)((a0n ^ (a0n >> 1)) & 1ull) : 0u;
      const uint32_t a1x = x1 ? (uint32_t)((a1n ^ (a1n >> 1)) & 1ull) : 0u;
      const uint32_t b0x = x1 ? (uint32_t)((b0n ^ (b0n >> 1)) & 1ull) : 0u;
      const uint32_t a0y = (uint32_t)((a0n ^ a1n) & 1ull);
      const uint32_t a1y = hy2 ? (uint32_t)((a1n ^ a2n) & 1ull) : 0u;
      auto own = [&](const Cross &k, uint32_t vb, uint32_t vbn, uint32_t bxn, uint32_t byn, int xo) {
        Owner o;
        if (xo < 64) {
          o.base = vb + (uint32_t)popc3_below(k, xo);
          o.bx = (uint32_t)((k.cx >> xo) & 1ull);
          o.by = (uint32_t)((k.cy >> xo) & 1ull);
        } else {
          o.base = vbn; o.bx = bxn; o.by = byn;
        }
        return o;
      };
      // the owner at i + 1 of the same row: the owner at i plus point i's
      // crossings (no second count of the row below it)
      auto next = [&](const Cross &k, const Owner &o, uint32_t vbn, uint32_t bxn, uint32_t byn) {
        Owner r;
        if (i + 1 < 64) {
          r.base = o.base + o.bx + o.by + (uint32_t)((k.cz >> i) & 1ull);
          r.bx = (uint32_t)((k.cx >> (i + 1)) & 1ull);
          r.by = (uint32_t)((k.cy >> (i + 1)) & 1ull);
        } else {
          r.base = vbn; r.bx = bxn; r.by = byn;
        }
        return r;
      };
      const Owner a00 = own(k0, v0, v0n, a0x, a0y, i);          // (dx,dy,dz) = (0,0,0)
      const Owner a10 = next(k0, a00, v0n, a0x, a0y);           // (1,0,0)
      const Owner b00 = own(k1, v1, v1n, a1x, a1y, i);          // (0,1,0)
      const Owner b10 = next(k1, b00, v1n, a1x, a1y);           // (1,1,0)
      const Owner d00 = own(k2, v2, v2n, b0x, 0u, i);           // (0,0,1)
      const Owner d10 = next(k2, d00, v2n, b0x, 0u);            // (1,0,1)
      const Owner e00 = own(k3, v3, v3, 0u, 0u, i);             // (0,1,1)
      // x edges 0..3 at (dy,dz) = (0,0), (1,0), (0,1), (1,1)
      my[0] = (int32_t)a00.base;
      my[1] = (int32_t)b00.base;
      my[2] = (int32_t)d00.base;
      my[3] = (int32_t)e00.base;
      // y edges 4..7 at (dx,dz) = (0,0), (1,0), (0,1), (1,1)
      my[4] = (int32_t)(a00.base + a00.bx);
      my[5] = (int32_t)(a10.base + a10.bx);
      my[6] = (int32_t)(d00.base + d00.bx);
      my[7] = (int32_t)(d10.base + d10.bx);
      // z edges 8..11 at (dx,dy) = (0,0), (1,0), (0,1), (1,1)
      my[8] = (int32_t)(a00.base + a00.bx + a00.by);
      my[9] = (int32_t)(a10.base + a10.bx + a10.by);
      my[10] = (int32_t)(b00.base + b00.bx + b00.by);
      my[11] = (int32_t)(b10.base + b10.bx + b10.by);
    }
    // the cell's offset in the workgroup's triangle range
    const u64 t0 = __ballot(nt & 1u), t1 = __ballot(nt & 2u), t2 = __ballot(nt & 4u);
    const uint32_t excl = lanes_below(t0) + 2 * lanes_below(t1) + 4 * lanes_below(t2);
    if (lane == 0) wsum[wave] = (uint32_t)(__popcll(t0) + 2 * __popcll(t1) + 4 * __popcll(t2));
    __syncthreads();
    uint32_t so = excl, total = 0;
#pragma unroll
    for (int w = 0; w < kWaves; w++) {
      so += (uint32_t)w < wave ? wsum[w] : 0u;
      total += wsum[w];
    }
    for (uint32_t t = 0; t < nt; t++)
      for (int q = 0; q < 3; q++) st[3 * (so + t) + q] = my[tab.tri[cs][3 * t + q]];
    __syncthreads();
    const uint32_t nint = 3 * total;
    const uint64_t capi = 3 * (uint64_t)M.cap_t;
    for (uint32_t q = threadIdx.x; q < nint; q += kBS) {
      const uint64_t g = 3 * (uint64_t)tbase + q;
      if (g < capi) M.tris[g] = st[q];
    }
    __syncthreads();
  }
}

__global__ void k_mc_counts(McPlan M, int with_lists) {
  if (threadIdx.x == 0) {
    const int64_t n = M.nrows * M.nw;
    M.counts[0] = (int64_t)M.P[n].x;
    M.counts[1] = (int64_t)M.P[n].y;
    if (with_lists) {
      M.counts[2] = (int64_t)M.P[n].z;
      M.counts[3] = (int64_t)M.P[n].w;
    }
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

static McPlan with_divisors(const McPlan &p) {
  McPlan q = p;
  q.d_nw = make_fastdiv((uint32_t)p.nw);
  q.d_n1 = make_fastdiv((uint32_t)p.n[1]);
  return q;
}

void launch_mc_count(const McPlan &p0, U4 *scan_tmp, hipStream_t s) {
  const McPlan p = with_divisors(p0);
  const int64_t nwords = p.nrows * p.nw;
  prof_mark("k_mc_bits", s, 0);
  k_mc_bits<<<dim3((unsigned)ceil_div(p.nrows, kWaves)), dim3(kBS), 0, s>>>(p);
  prof_mark("k_mc_bits", s, 1);
  prof_mark("k_mc_count", s, 0);
  k_mc_count<<<dim3((unsigned)ceil_div(nwords, kBS)), dim3(kBS), 0, s>>>(p);
  prof_mark("k_mc_count", s, 1);
  scan_u4_packed(p.cnt, p.P, nwords, scan_tmp, s);
  k_mc_counts<<<dim3(1), dim3(64), 0, s>>>(p, 1);
}

void launch_mc_emit(const McPlan &p0, hipStream_t s) {
  const McPlan p = with_divisors(p0);
  const int64_t nwords = p.nrows * p.nw;
  prof_mark("k_mc_expand", s, 0);
  k_mc_expand<<<dim3((unsigned)ceil_div(nwords, kBS)), dim3(kBS), 0, s>>>(p);
  prof_mark("k_mc_expand", s, 1);
  // list lengths live on the device: a fixed grid strides over them
  prof_mark("k_mc_verts", s, 0);
  k_mc_verts<<<dim3(2048), dim3(kBS), 0, s>>>(p);
  prof_mark("k_mc_verts", s, 1);
  prof_mark("k_mc_tris", s, 0);
  k_mc_tris<<<dim3(2048), dim3(kBS), 0, s>>>(p);
  prof_mark("k_mc_tris", s, 1);
}

void launch_mc(const McPlan &p0, U4 *scan_tmp, hipStream_t s) {
  const McPlan p = with_divisors(p0);
  const int64_t nwords = p.nrows * p.nw;
  prof_mark("k_mc_bits", s, 0);
  k_mc_bits<<<dim3((unsigned)ceil_div(p.nrows, kWaves)), dim3(kBS), 0, s>>>(p);
  prof_mark("k_mc_bits", s, 1);
  prof_mark("k_mc_count", s, 0);
  k_mc_count<<<dim3((unsigned)ceil_div(nwords, kBS)), dim3(kBS), 0, s>>>(p);
  prof_mark("k_mc_count", s, 1);
  scan_u4_packed(p.cnt, p.P, nwords, scan_tmp, s);
  launch_mc_emit(p, s);
}

void launch_mc_bits(const McPlan &p0, hipStream_t s) {
  const McPlan p = with_divisors(p0);
  prof_mark("k_mc_bits", s, 0);
  k_mc_bits<<<dim3((unsigned)ceil_div(p.nrows, kWaves)), dim3(kBS), 0, s>>>(p);
  prof_mark("k_mc_bits", s, 1);
}

void launch_mc_from_bits(const McPlan &p0, U4 *scan_tmp, hipStream_t s) {
  const McPlan p = with_divisors(p0);
  const int64_t nwords = p.nrows * p.nw;
  prof_mark("k_mc_count", s, 0);
  k_mc_count<<<dim3((unsigned)ceil_div(nwords, kBS)), dim3(kBS), 0, s>>>(p);
  prof_mark("k_mc_count", s, 1);
  scan_u4_packed(p.cnt, p.P, nwords, scan_tmp, s);
  launch_mc_emit(p, s);
}

void launch_mc_cases(const McPlan &p0, hipStream_t s) {
  const McPlan p = with_divisors(p0);
  const int64_t nwords = p.nrows * p.nw;
  k_mc_bits<<<dim3((unsigned)ceil_div(p.nrows, kWaves)), dim3(kBS), 0, s>>>(p);
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
