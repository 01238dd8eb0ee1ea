// topo.hip -- the paper's error translation for topology preservation
// (Sec. II.B): over every grid edge whose end values s0 < s1 enclose an
// isovalue k strictly (s0 < k < s1), the distances d0 = k - s0 and
// d1 = s1 - k form the multiset D; an error bound below min(D) keeps every
// crossing, and the n-th smallest entry of D relaxes it (topology accuracy
// below 100%).
//
// D is never materialized.  Every pass recomputes the entries from the
// field (one wave per 64 points of a row, the four loads of a point's +x/+y/+z
// edges coalesced) and feeds them to one of: a count, a minimum, or one
// 8-bit digit of a most-significant-digit radix select.  Entries are
// positive doubles, whose bit patterns order as unsigned integers, so the
// select works on the 64-bit patterns; the state between passes stays on the
// device.
#include <algorithm>

#include "chr_plan.h"

namespace chr {
namespace {

constexpr int kBS = 256;
constexpr int kWaves = kBS / kWave;
constexpr int kUnroll = 4;   // words in flight per wave

struct TopoState {
  unsigned long long total;   // |D|
  unsigned long long minkey;  // smallest entry (bits)
  unsigned long long prefix;  // selected high digits so far
  unsigned long long mask;    // which bits of prefix are fixed
  unsigned long long nrem;    // rank (1-based) still to find below the prefix
  unsigned long long hist[256];
};

struct TopoPlan {
  const float *f;
  int64_t n[3];
  int K;
  float iso[kMaxIso];
  TopoState *st;
  double *out;       // {bound, |D|}
  int64_t nth;
  uint32_t nw;       // 64-point words per row
  FastDiv d_nw, d_n1;
};

// mode 0: count and minimum; 2: histogram of digit `shift` among entries
// matching the prefix.  One wave per row of points (grid-stride), 64
// consecutive points per step; crossings are tested in binary32 (exact:
// the isovalue and the end values are binary32) and only crossing edges form
// their double distances.
template <int MODE>
__global__ __launch_bounds__(kBS) void k_topo_pass(TopoPlan T, int shift) {
  __shared__ unsigned int hist[256];
  if (MODE == 2) {
    for (int i = threadIdx.x; i < 256; i += kBS) hist[i] = 0u;
    __syncthreads();
  }
  const int lane = lane_id();
  const uint32_t n0 = (uint32_t)T.n[0], n1 = (uint32_t)T.n[1], n2 = (uint32_t)T.n[2];
  const uint32_t nrows = n0 * n1;
  const size_t plane = (size_t)n1 * n2;
  const unsigned long long prefix = (MODE == 2) ? T.st->prefix : 0ull, mask = (MODE == 2) ? T.st->mask : 0ull;
  const int K = T.K;
  unsigned long long cnt = 0, kmin = ~0ull;
  auto take = [&](unsigned long long e) {
    if (MODE == 0) {
      cnt++;
      kmin = min(kmin, e);
    } else if ((e & mask) == prefix) {
      atomicAdd(&hist[(e >> shift) & 255u], 1u);
    }
  };
  // consecutive waves take consecutive 64-point words, so the rows above
  // (+y) and the plane above (+z) that a word reads are fetched by waves
  // running at the same time; each wave issues the loads of kUnroll words
  // (spaced by the grid's wave count) before using any of them
  const uint32_t nwords = nrows * T.nw;
  const uint32_t nwaves = gridDim.x * kWaves;
  for (uint32_t g0 = blockIdx.x * kWaves + threadIdx.x / kWave; g0 < nwords; g0 += nwaves * kUnroll) {
    float v[kUnroll][4];
    uint32_t yy[kUnroll], zz[kUnroll], xx[kUnroll];
    bool on[kUnroll];
#pragma unroll
    for (int q = 0; q < kUnroll; q++) {
      const uint32_t gw = g0 + (uint32_t)q * nwaves;
      const uint32_t row = fdiv(gw < nwords ? gw : 0u, T.d_nw);
      const uint32_t x = (gw - row * T.nw) * 64u + (uint32_t)lane;
      on[q] = gw < nwords && x < n2;
      const uint32_t z = fdiv(row, T.d_n1), y = row - z * n1;
      const bool hx = x + 1 < n2, hy = y + 1 < n1, hz = z + 1 < n0;
      const uint32_t xs = on[q] ? x : 0u;
      // four independent loads; a missing neighbour reads the point itself,
      // which encloses nothing
      const float *__restrict__ fr = T.f + (size_t)row * n2;
      v[q][0] = fr[xs];
      v[q][1] = fr[(on[q] && hx) ? xs + 1 : xs];
      v[q][2] = fr[(on[q] && hy) ? xs + n2 : xs];
      v[q][3] = fr[(on[q] && hz) ? xs + plane : xs];
      xx[q] = x; yy[q] = y; zz[q] = z;
    }
#pragma unroll
    for (int q = 0; q < kUnroll; q++) {
      if (!on[q]) continue;
      const float s = v[q][0];
      for (int j = 0; j < K; j++) {
        const float k = T.iso[j];
#pragma unroll
        for (int a = 1; a <= 3; a++) {
          const float sn = v[q][a];
          const float lo = fminf(s, sn), hi = fmaxf(s, sn);
          if (lo < k && k < hi) {
            const double kd = (double)k;
            take((unsigned long long)__double_as_longlong(kd - (double)lo));
            take((unsigned long long)__double_as_longlong((double)hi - kd));
          }
        }
      }
    }
    (void)xx; (void)yy; (void)zz;
  }
  if (MODE == 0) {
    for (int m = 32; m >= 1; m >>= 1) {
      cnt += __shfl_xor(cnt, m, kWave);
      kmin = min(kmin, (unsigned long long)__shfl_xor(kmin, m, kWave));
    }
    if (lane == 0 && cnt) {
      atomicAdd(&T.st->total, cnt);
      atomicMin(&T.st->minkey, kmin);
    }
  }
  if (MODE == 2) {
    __syncthreads();
    for (int i = threadIdx.x; i < 256; i += kBS)
      if (hist[i]) atomicAdd(&T.st->hist[i], (unsigned long long)hist[i]);
  }
}

// Resets the state (a kernel, so that the whole computation can be captured).
__global__ void k_topo_init(TopoPlan T) {
  TopoState *st = T.st;
  for (int i = threadIdx.x; i < 256; i += blockDim.x) st->hist[i] = 0ull;
  if (threadIdx.x == 0) {
    st->total = 0ull;
    st->minkey = ~0ull;
    st->prefix = 0ull;
    st->mask = 0ull;
    st->nrem = 0ull;
  }
}

// After the count: the rank to find, clamped to [1, |D|].
__global__ void k_topo_rank(TopoPlan T) {
  if (threadIdx.x != 0) return;
  TopoState *st = T.st;
  const unsigned long long m = st->total;
  unsigned long long n = T.nth < 1 ? 1ull : (unsigned long long)T.nth;
  if (n > m) n = m;
  st->nrem = n;
}

// After a histogram pass: fixes the digit holding the rank-th entry, and
// clears the histogram for the next pass.
__global__ void k_topo_digit(TopoPlan T, int shift) {
  if (threadIdx.x != 0) return;
  TopoState *st = T.st;
  if (st->total == 0) return;
  unsigned long long below = 0;
  int bin = 255;
  for (int i = 0; i < 256; i++) {
    if (below + st->hist[i] >= st->nrem) { bin = i; break; }
    below += st->hist[i];
  }
  st->nrem -= below;
  st->prefix |= (unsigned long long)bin << shift;
  st->mask |= 255ull << shift;
  for (int i = 0; i < 256; i++) st->hist[i] = 0ull;
}

__global__ void k_topo_finish(TopoPlan T, int selected) {
  if (threadIdx.x != 0) return;
  const TopoState *st = T.st;
  double r = __longlong_as_double(0x7ff0000000000000ll);  // +inf: no crossing edge
  if (st->total) r = __longlong_as_double((long long)(selected ? st->prefix : st->minkey));
  T.out[0] = r;
  T.out[1] = (double)st->total;
}

}  // namespace

size_t topo_workspace_bytes() { return sizeof(TopoState); }

int launch_topology(const float *f, const int64_t dims[3], const float *iso, int K, int64_t nth, double *out,
                    void *ws, hipStream_t s) {
  TopoPlan T;
  T.f = f;
  for (int a = 0; a < 3; a++) T.n[a] = dims[a];
  T.K = K;
  for (int j = 0; j < kMaxIso; j++) T.iso[j] = j < K ? iso[j] : 0.f;
  T.st = static_cast<TopoState *>(ws);
  T.out = out;
  T.nth = nth;
  T.nw = (uint32_t)ceil_div(dims[2], 64);
  T.d_nw = make_fastdiv(T.nw);
  T.d_n1 = make_fastdiv((uint32_t)dims[1]);
  const int64_t nwords = dims[0] * dims[1] * (int64_t)T.nw;
  // about one resident wave per SIMD slot; each wave loops over its words
  const int64_t grid = std::min<int64_t>(std::max<int64_t>(ceil_div(nwords, (int64_t)kWaves * kUnroll), 1), 2048);
  k_topo_init<<<1, 256, 0, s>>>(T);
  k_topo_pass<0><<<dim3((unsigned)grid), dim3(kBS), 0, s>>>(T, 0);  // |D| and min(D)
  const bool select = nth > 1;
  if (select) {
    k_topo_rank<<<1, 64, 0, s>>>(T);
    for (int shift = 56; shift >= 0; shift -= 8) {
      k_topo_pass<2><<<dim3((unsigned)grid), dim3(kBS), 0, s>>>(T, shift);
      k_topo_digit<<<1, 64, 0, s>>>(T, shift);
    }
  }
  k_topo_finish<<<1, 64, 0, s>>>(T, select ? 1 : 0);
  return 0;
}

}  // namespace chr
