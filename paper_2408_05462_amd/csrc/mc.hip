// mc.hip -- marching cubes on gfx950 (Sec. I: isosurface generation;
// Sec. II.B: the per-cell case that topology preservation keeps).
//
//  1. k_mc_bits:  one coalesced pass over the field; a wave ballots f < k for
//     64 consecutive points of a row and stores the 64-bit word (1 bit/point).
//  2. k_mc_count: one wave per row of points; from the bit rows (y,z),
//     (y+1,z), (y,z+1), (y+1,z+1) it counts the row's crossing owned edges
//     (+x,+y,+z of each point) with popcounts on wave-uniform words, and the
//     triangles of the cell row (case per lane, table lookup, wave sum).
//  3. scan of the per-row counts (vertex and triangle offsets).
//  4. k_mc_emit:  one wave per active row; vertex ids come from the row
//     offsets plus popcounts of the crossing masks below a point, so every
//     triangle finds its three vertex ids without any per-point id array.
//     Vertices are interpolated at t = (k - fa) / (fb - fa).
#include "chr_plan.h"
#include "mc_table.h"

namespace chr {
namespace {

constexpr int kBS = 256;
constexpr int kWaves = kBS / kWave;

constexpr mct::Table kTable = mct::make_table();
__constant__ mct::Table c_table = kTable;

__global__ __launch_bounds__(kBS) void k_mc_bits(McPlan M) {
  const int64_t nwords = M.nrows * M.nw;
  const int64_t wid = (int64_t)blockIdx.x * kWaves + threadIdx.x / kWave;
  if (wid >= nwords) return;
  const int64_t row = wid / M.nw, w = wid % M.nw;
  const int64_t x = w * 64 + lane_id();
  bool below = false;
  if (x < M.n[2]) below = M.f[row * M.n[2] + x] < M.k;
  const unsigned long long m = __ballot(below);
  if (lane_id() == 0) M.bits[wid] = m;
}

// Crossing masks of the owned +x/+y/+z edges of word w of point row (y, z).
struct Cross {
  unsigned long long cx, cy, cz;
};

__device__ inline Cross cross_masks(const McPlan &M, int64_t z, int64_t y, int64_t w) {
  Cross c{0, 0, 0};
  if (w < 0 || w >= M.nw || y >= M.n[1] || z >= M.n[0]) return c;
  const int64_t r = z * M.n[1] + y;
  const unsigned long long *B = M.bits;
  const unsigned long long m = B[r * M.nw + w];
  const unsigned long long nx = (w + 1 < M.nw) ? B[r * M.nw + w + 1] : 0ull;
  const int64_t nxp = M.n[2];
  const int64_t rem = nxp - w * 64;  // valid points in this word
  const unsigned long long valid = rem >= 64 ? ~0ull : ((1ull << rem) - 1ull);
  // +x edges exist for points x + 1 < nx
  const int64_t remx = rem - 1;
  const unsigned long long validx = remx >= 64 ? ~0ull : (remx <= 0 ? 0ull : ((1ull << remx) - 1ull));
  c.cx = (m ^ ((m >> 1) | (nx << 63))) & validx;
  if (y + 1 < M.n[1]) c.cy = (m ^ B[(r + 1) * M.nw + w]) & valid;
  if (z + 1 < M.n[0]) c.cz = (m ^ B[(r + M.n[1]) * M.nw + w]) & valid;
  return c;
}

__device__ inline unsigned long long shifted(const unsigned long long *B, int64_t base, int64_t w, int64_t nw) {
  const unsigned long long m = B[base + w];
  const unsigned long long nx = (w + 1 < nw) ? B[base + w + 1] : 0ull;
  return (m >> 1) | (nx << 63);
}

// Case of the cell at this lane from the four bit rows of the cell row.
__device__ inline uint32_t cell_case(unsigned long long m00, unsigned long long s00, unsigned long long m10,
                                     unsigned long long s10, unsigned long long m01, unsigned long long s01,
                                     unsigned long long m11, unsigned long long s11, int lane) {
  return (uint32_t)(((m00 >> lane) & 1) | (((s00 >> lane) & 1) << 1) | (((m10 >> lane) & 1) << 2) |
                    (((s10 >> lane) & 1) << 3) | (((m01 >> lane) & 1) << 4) | (((s01 >> lane) & 1) << 5) |
                    (((m11 >> lane) & 1) << 6) | (((s11 >> lane) & 1) << 7));
}

__global__ __launch_bounds__(kBS) void k_mc_count(McPlan M) {
  const int64_t row = (int64_t)blockIdx.x * kWaves + threadIdx.x / kWave;
  if (row >= M.nrows) return;
  const int lane = lane_id();
  const int64_t z = row / M.n[1], y = row % M.n[1];
  const bool cells = (y + 1 < M.n[1]) && (z + 1 < M.n[0]);
  uint32_t nv = 0, nt = 0;
  const unsigned long long *B = M.bits;
  for (int64_t w = 0; w < M.nw; w++) {
    const Cross c = cross_masks(M, z, y, w);
    nv += (uint32_t)(__popcll(c.cx) + __popcll(c.cy) + __popcll(c.cz));
    if (cells) {
      const int64_t r00 = row * M.nw, r10 = (row + 1) * M.nw, r01 = (row + M.n[1]) * M.nw,
                    r11 = (row + M.n[1] + 1) * M.nw;
      const uint32_t cs = cell_case(B[r00 + w], shifted(B, r00, w, M.nw), B[r10 + w], shifted(B, r10, w, M.nw),
                                    B[r01 + w], shifted(B, r01, w, M.nw), B[r11 + w], shifted(B, r11, w, M.nw), lane);
      const int64_t x = w * 64 + lane;
      nt += (x + 1 < M.n[2]) ? c_table.ntri[cs] : 0u;
    }
  }
  nt = wave_sum_u(nt);
  if (lane == 0) M.cnt[row] = U4{nv, nt, 0u, 0u};
}

__device__ inline float interp(float fa, float fb, float k) {
  return __fdiv_rn(__fsub_rn(k, fa), __fsub_rn(fb, fa));
}

__global__ __launch_bounds__(kBS) void k_mc_emit(McPlan M) {
  const int64_t row = (int64_t)blockIdx.x * kWaves + threadIdx.x / kWave;
  if (row >= M.nrows) return;
  const U4 p0 = M.P[row], p1 = M.P[row + 1];
  const uint32_t nv_row = p1.x - p0.x, nt_row = p1.y - p0.y;
  if (nv_row == 0 && nt_row == 0) return;
  const int lane = lane_id();
  const unsigned long long below_lane = (1ull << lane) - 1ull;
  const int64_t z = row / M.n[1], y = row % M.n[1];
  const int64_t n1 = M.n[1], n2 = M.n[2];
  const float *f = M.f;
  const float k = M.k, sp = M.spacing;

  // vertices of this point row
  if (nv_row) {
    uint64_t run = p0.x;
    for (int64_t w = 0; w < M.nw; w++) {
      const Cross c = cross_masks(M, z, y, w);
      const uint32_t tot = (uint32_t)(__popcll(c.cx) + __popcll(c.cy) + __popcll(c.cz));
      if (tot) {
        const int64_t x = w * 64 + lane;
        uint64_t id = run + (uint64_t)(__popcll(c.cx & below_lane) + __popcll(c.cy & below_lane) +
                                       __popcll(c.cz & below_lane));
        const bool ex = (c.cx >> lane) & 1, ey = (c.cy >> lane) & 1, ez = (c.cz >> lane) & 1;
        if (ex || ey || ez) {
          const float fa = f[(z * n1 + y) * n2 + x];
          const float px = (float)x, py = (float)y, pz = (float)z;
          if (ex) {
            if ((int64_t)id < M.cap_v) {
              const float t = interp(fa, f[(z * n1 + y) * n2 + x + 1], k);
              float *v = M.verts + 3 * id;
              v[0] = __fmul_rn(__fadd_rn(px, t), sp); v[1] = __fmul_rn(py, sp); v[2] = __fmul_rn(pz, sp);
            }
            id++;
          }
          if (ey) {
            if ((int64_t)id < M.cap_v) {
              const float t = interp(fa, f[(z * n1 + y + 1) * n2 + x], k);
              float *v = M.verts + 3 * id;
              v[0] = __fmul_rn(px, sp); v[1] = __fmul_rn(__fadd_rn(py, t), sp); v[2] = __fmul_rn(pz, sp);
            }
            id++;
          }
          if (ez) {
            if ((int64_t)id < M.cap_v) {
              const float t = interp(fa, f[((z + 1) * n1 + y) * n2 + x], k);
              float *v = M.verts + 3 * id;
              v[0] = __fmul_rn(px, sp); v[1] = __fmul_rn(py, sp); v[2] = __fmul_rn(__fadd_rn(pz, t), sp);
            }
            id++;
          }
        }
      }
      run += tot;
    }
  }

  // triangles of this cell row
  if (nt_row) {
    const unsigned long long *B = M.bits;
    const int64_t rows[4] = {row, row + 1, row + n1, row + n1 + 1};   // owner rows (dy,dz) = 00,10,01,11
    const int64_t ry[4] = {y, y + 1, y, y + 1}, rz[4] = {z, z, z + 1, z + 1};
    uint64_t vbase[4];
    for (int i = 0; i < 4; i++) vbase[i] = M.P[rows[i]].x;
    uint64_t trun = p0.y;
    Cross cur[4], nxt[4];
    for (int i = 0; i < 4; i++) cur[i] = cross_masks(M, rz[i], ry[i], 0);
    for (int64_t w = 0; w < M.nw; w++) {
      for (int i = 0; i < 4; i++) nxt[i] = cross_masks(M, rz[i], ry[i], w + 1);
      const int64_t r00 = row * M.nw, r10 = (row + 1) * M.nw, r01 = (row + n1) * M.nw, r11 = (row + n1 + 1) * M.nw;
      const uint32_t cs = cell_case(B[r00 + w], shifted(B, r00, w, M.nw), B[r10 + w], shifted(B, r10, w, M.nw),
                                    B[r01 + w], shifted(B, r01, w, M.nw), B[r11 + w], shifted(B, r11, w, M.nw), lane);
      const int64_t x = w * 64 + lane;
      const uint32_t ntr = (x + 1 < n2) ? c_table.ntri[cs] : 0u;
      const uint32_t toff = wave_excl_sum(ntr);
      for (uint32_t t = 0; t < ntr; t++) {
        const uint64_t tid = trun + toff + t;
        int32_t ids[3];
        for (int q = 0; q < 3; q++) {
          const int e = c_table.tri[cs][3 * t + q];
          const int axis = e >> 2, i2 = e & 3;
          // owner point of the edge: cell origin + the edge's lower corner
          int dx = 0, dy = 0, dz = 0;
          if (axis == 0) { dy = i2 & 1; dz = i2 >> 1; }
          if (axis == 1) { dx = i2 & 1; dz = i2 >> 1; }
          if (axis == 2) { dx = i2 & 1; dy = i2 >> 1; }
          const int R = dy + 2 * dz;
          const int xi = lane + dx;  // 0..64 within this word
          Cross cw;
          unsigned long long bm;
          int bit;
          if (xi < 64) { cw = cur[R]; bm = (1ull << xi) - 1ull; bit = xi; }
          else { cw = nxt[R]; bm = 0ull; bit = 0; }
          uint64_t before = (xi < 64) ? (uint64_t)(__popcll(cw.cx & bm) + __popcll(cw.cy & bm) + __popcll(cw.cz & bm))
                                      : (uint64_t)(__popcll(cur[R].cx) + __popcll(cur[R].cy) + __popcll(cur[R].cz));
          uint64_t within = 0;
          if (axis >= 1) within += (cw.cx >> bit) & 1;
          if (axis >= 2) within += (cw.cy >> bit) & 1;
          ids[q] = (int32_t)(vbase[R] + before + within);
        }
        if ((int64_t)tid < M.cap_t) {
          int32_t *o = M.tris + 3 * tid;
          o[0] = ids[0]; o[1] = ids[1]; o[2] = ids[2];
        }
      }
      trun += wave_sum_u(ntr);
      for (int i = 0; i < 4; i++) {
        vbase[i] += (uint64_t)(__popcll(cur[i].cx) + __popcll(cur[i].cy) + __popcll(cur[i].cz));
        cur[i] = nxt[i];
      }
    }
  }
}

__global__ void k_mc_counts(McPlan M) {
  if (threadIdx.x == 0) {
    M.counts[0] = (int64_t)M.P[M.nrows].x;
    M.counts[1] = (int64_t)M.P[M.nrows].y;
  }
}

__global__ __launch_bounds__(kBS) void k_mc_cases(McPlan M) {
  const int64_t cz = M.n[0] - 1, cy = M.n[1] - 1, cx = M.n[2] - 1;
  const int64_t row = (int64_t)blockIdx.x * kWaves + threadIdx.x / kWave;
  if (row >= cz * cy) return;
  const int lane = lane_id();
  const int64_t z = row / cy, y = row % cy;
  const int64_t prow = z * M.n[1] + y;
  const unsigned long long *B = M.bits;
  for (int64_t w = 0; w < M.nw; w++) {
    const int64_t r00 = prow * M.nw, r10 = (prow + 1) * M.nw, r01 = (prow + M.n[1]) * M.nw,
                  r11 = (prow + M.n[1] + 1) * M.nw;
    const uint32_t cs = cell_case(B[r00 + w], shifted(B, r00, w, M.nw), B[r10 + w], shifted(B, r10, w, M.nw),
                                  B[r01 + w], shifted(B, r01, w, M.nw), B[r11 + w], shifted(B, r11, w, M.nw), lane);
    const int64_t x = w * 64 + lane;
    if (x < cx) M.cases[(z * cy + y) * cx + x] = (uint8_t)cs;
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
  k_mc_bits<<<dim3((unsigned)ceil_div(nwords, kWaves)), dim3(kBS), 0, s>>>(p);
  prof_mark("k_mc_bits", s, 1);
  prof_mark("k_mc_count", s, 0);
  k_mc_count<<<dim3((unsigned)ceil_div(p.nrows, kWaves)), dim3(kBS), 0, s>>>(p);
  prof_mark("k_mc_count", s, 1);
  scan_u4(p.cnt, p.P, p.nrows, scan_tmp, s);
  prof_mark("k_mc_emit", s, 0);
  k_mc_emit<<<dim3((unsigned)ceil_div(p.nrows, kWaves)), dim3(kBS), 0, s>>>(p);
  prof_mark("k_mc_emit", s, 1);
  k_mc_counts<<<dim3(1), dim3(64), 0, s>>>(p);
}

void launch_mc_cases(const McPlan &p, hipStream_t s) {
  const int64_t nwords = p.nrows * p.nw;
  prof_mark("k_mc_bits", s, 0);
  k_mc_bits<<<dim3((unsigned)ceil_div(nwords, kWaves)), dim3(kBS), 0, s>>>(p);
  prof_mark("k_mc_bits", s, 1);
  const int64_t crow = (p.n[0] - 1) * (p.n[1] - 1);
  if (crow > 0 && p.n[2] > 1) k_mc_cases<<<dim3((unsigned)ceil_div(crow, kWaves)), dim3(kBS), 0, s>>>(p);
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
