// scan.hip -- device-wide exclusive prefix sums for gfx950.
//
// Three launches: per-tile totals (coalesced loads, all in flight together),
// one workgroup scanning the tile totals, and a downsweep.  For the 4 x u32
// records (the chunk and word counts) a wave scans its 512 consecutive
// elements as 8 rows of 64 with DPP (row shifts, then row broadcasts), so a
// tile needs one workgroup barrier; the 64-bit scans (short: section sizes)
// keep the shuffle-based block scan.  Small inputs take one launch.
#include "scan.h"

#include <type_traits>

#include "chr_device.h"

namespace chr {
namespace {

constexpr int kBS = 256;
constexpr int kIPT = 8;
constexpr int kTile = kBS * kIPT;
constexpr int64_t kFuseTiles = 2048;  // 4 x u32 scans of at most this many tiles skip the tile-total scan

template <class T> __device__ inline T zero();
template <> __device__ inline U4 zero<U4>() { return U4{0, 0, 0, 0}; }
template <> __device__ inline uint64_t zero<uint64_t>() { return 0; }

__device__ inline U4 add(U4 a, U4 b) { return U4{a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w}; }
__device__ inline uint64_t add(uint64_t a, uint64_t b) { return a + b; }
__device__ inline U4 sub(U4 a, U4 b) { return U4{a.x - b.x, a.y - b.y, a.z - b.z, a.w - b.w}; }
__device__ inline uint64_t sub(uint64_t a, uint64_t b) { return a - b; }

__device__ inline U4 shfl_up_t(U4 v, int d) {
  return U4{__shfl_up(v.x, d, kWave), __shfl_up(v.y, d, kWave), __shfl_up(v.z, d, kWave),
            __shfl_up(v.w, d, kWave)};
}
__device__ inline uint64_t shfl_up_t(uint64_t v, int d) { return __shfl_up(v, d, kWave); }

// Exclusive scan over the 256 threads of a workgroup; *total = sum of all.
template <class T>
__device__ T block_excl_scan(T v, T *total, T *lds) {
  const int lid = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  T x = v;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    T y = shfl_up_t(x, d);
    if (lid >= d) x = add(x, y);
  }
  if (lid == kWave - 1) lds[wid] = x;
  __syncthreads();
  T pre = zero<T>(), tot = zero<T>();
#pragma unroll
  for (int w = 0; w < kBS / kWave; w++) {
    if (w < wid) pre = add(pre, lds[w]);
    tot = add(tot, lds[w]);
  }
  __syncthreads();
  *total = tot;
  return add(pre, sub(x, v));
}

// Inclusive sum over the 64 lanes through DPP: shifts by 1, 2, 4 and 8
// within each 16-lane row, then the broadcasts of lanes 15 and 31 into the
// rows after them (a lane without a source adds 0).
__device__ inline uint32_t wave_incl_u32(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);   // row_shr:1
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);   // row_shr:2
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);   // row_shr:4
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);   // row_shr:8
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);   // row_bcast:15
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);   // row_bcast:31
  return v;
}
__device__ inline U4 wave_incl(U4 v) {
  return U4{wave_incl_u32(v.x), wave_incl_u32(v.y), wave_incl_u32(v.z), wave_incl_u32(v.w)};
}
__device__ inline U4 lane63(U4 v) {
  return U4{(uint32_t)__builtin_amdgcn_readlane((int)v.x, 63), (uint32_t)__builtin_amdgcn_readlane((int)v.y, 63),
            (uint32_t)__builtin_amdgcn_readlane((int)v.z, 63), (uint32_t)__builtin_amdgcn_readlane((int)v.w, 63)};
}

// Records as scanned: 4 x u32 as stored, or unpacked from the 32-bit form
// of marching cubes' word counts (see scan.h).
__device__ inline U4 rec(const U4 *in, int64_t k) { return in[k]; }
__device__ inline U4 rec(const uint32_t *in, int64_t k) {
  const uint32_t c = in[k];
  return U4{c & 0xffu, (c >> 8) & 0x1ffu, (c >> 17) & 0x7fu, (c >> 24) & 0x7fu};
}

// The lane's kIPT records of a wave's run (zeros past n; n >= 1 here), all
// loads in flight together: each load is clamped and its record masked by
// an opaque mask, as with a select the compiler moves every load into a
// branch and waits for it there.
template <class In>
__device__ __forceinline__ void load_recs(const In *__restrict__ in, int64_t base, int lane, int64_t n,
                                          U4 (&v)[kIPT]) {
  uint32_t m[kIPT];
#pragma unroll
  for (int r = 0; r < kIPT; r++) {
    m[r] = base + r * kWave + lane < n ? ~0u : 0u;
    asm volatile("" : "+v"(m[r]));
  }
#pragma unroll
  for (int r = 0; r < kIPT; r++) {
    const int64_t k = base + r * kWave + lane;
    const U4 x = rec(in, k < n ? k : n - 1);
    v[r] = U4{x.x & m[r], x.y & m[r], x.z & m[r], x.w & m[r]};
  }
}

// Tile totals of 4 x u32 records: eight loads a lane, a DPP sum per wave.
template <class In>
__global__ __launch_bounds__(kBS) void k_scan_reduce_u4(const In *__restrict__ in, U4 *__restrict__ part, int64_t n) {
  __shared__ U4 lds[kBS / kWave];
  const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)(threadIdx.x / kWave) * (kTile / (kBS / kWave));
  const int lane = (int)(threadIdx.x & (kWave - 1));
  U4 v[kIPT];
  load_recs(in, base, lane, n, v);
  U4 t = U4{0, 0, 0, 0};
#pragma unroll
  for (int r = 0; r < kIPT; r++) t = add(t, v[r]);
  t = lane63(wave_incl(t));
  if (lane == 0) lds[threadIdx.x / kWave] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    U4 tot = lds[0];
#pragma unroll
    for (int w = 1; w < kBS / kWave; w++) tot = add(tot, lds[w]);
    part[blockIdx.x] = tot;
  }
}

// Downsweep of 4 x u32 records: a wave's 512 consecutive elements as 8 rows
// of 64 (DPP scans with a running carry), the waves' totals through LDS
// (one barrier), the tile's prefix from the partials.
// FROM_TOTALS: the tile's prefix is summed here from the tile totals before
// it (each thread a strided share, reduced with the waves' run totals
// through the same barrier), instead of read from a scanned array; the last
// tile writes the grand total to out[n].  For up to kFuseTiles tiles, where
// that costs less than a separate launch.
template <class In, bool FROM_TOTALS = false>
__global__ __launch_bounds__(kBS) void k_scan_down_u4(const In *__restrict__ in, U4 *__restrict__ out,
                                                      const U4 *__restrict__ part, int64_t n) {
  __shared__ U4 lds[kBS / kWave];
  __shared__ U4 ldp[kBS / kWave];
  const uint32_t wave = threadIdx.x / kWave;
  const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)wave * (kTile / (kBS / kWave));
  const int lane = (int)(threadIdx.x & (kWave - 1));
  U4 v[kIPT];
  load_recs(in, base, lane, n, v);
  U4 carry = U4{0, 0, 0, 0};
#pragma unroll
  for (int r = 0; r < kIPT; r++) {
    const U4 inc = add(wave_incl(v[r]), carry);
    carry = lane63(inc);
    v[r] = sub(inc, v[r]);                     // exclusive within the wave's run
  }
  U4 pre;
  if (FROM_TOTALS) {
    U4 t = U4{0, 0, 0, 0};
    // four totals per thread in flight (clamped loads, masked adds)
    for (uint32_t i0 = threadIdx.x; i0 < blockIdx.x; i0 += 4 * kBS) {
      U4 q[4];
#pragma unroll
      for (int j = 0; j < 4; j++) q[j] = part[min(i0 + (uint32_t)j * kBS, blockIdx.x - 1)];
#pragma unroll
      for (int j = 0; j < 4; j++)
        if (i0 + (uint32_t)j * kBS < blockIdx.x) t = add(t, q[j]);
    }
    t = lane63(wave_incl(t));
    if (lane == 0) {
      lds[wave] = carry;
      ldp[wave] = t;
    }
    __syncthreads();
    pre = add(add(ldp[0], ldp[1]), add(ldp[2], ldp[3]));
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0)
      out[n] = add(pre, add(add(lds[0], lds[1]), add(lds[2], lds[3])));
  } else {
    if (lane == 0) lds[wave] = carry;
    __syncthreads();
    pre = part[blockIdx.x];
  }
  for (uint32_t w = 0; w < wave; w++) pre = add(pre, lds[w]);
#pragma unroll
  for (int r = 0; r < kIPT; r++) {
    const int64_t k = base + r * kWave + lane;
    if (k < n) out[k] = add(pre, v[r]);
  }
}

template <class T>
__global__ __launch_bounds__(kBS) void k_scan_reduce(const T *__restrict__ in, T *__restrict__ part, int64_t n) {
  __shared__ T lds[kBS / kWave];
  const int64_t base = (int64_t)blockIdx.x * kTile;
  T s = zero<T>();
#pragma unroll
  for (int i = 0; i < kIPT; i++) {
    int64_t k = base + i * kBS + threadIdx.x;
    if (k < n) s = add(s, in[k]);
  }
  T tot;
  block_excl_scan(s, &tot, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

template <class T>
__global__ __launch_bounds__(kBS) void k_scan_part(T *__restrict__ part, int64_t ntiles, T *__restrict__ out_total) {
  __shared__ T lds[kBS / kWave];
  T carry = zero<T>();
  for (int64_t b = 0; b < ntiles; b += kBS) {
    int64_t k = b + threadIdx.x;
    T v = k < ntiles ? part[k] : zero<T>();
    T tot;
    T ex = block_excl_scan(v, &tot, lds);
    if (k < ntiles) part[k] = add(carry, ex);
    carry = add(carry, tot);
  }
  if (threadIdx.x == 0) *out_total = carry;
}

template <class T>
__global__ __launch_bounds__(kBS) void k_scan_down(const T *__restrict__ in, T *__restrict__ out,
                                                   const T *__restrict__ part, int64_t n) {
  __shared__ T lds[kBS / kWave];
  const int64_t base = (int64_t)blockIdx.x * kTile;
  T carry = part[blockIdx.x];
  for (int i = 0; i < kIPT; i++) {
    int64_t k = base + i * kBS + threadIdx.x;
    T v = k < n ? in[k] : zero<T>();
    T tot;
    T ex = block_excl_scan(v, &tot, lds);
    if (k < n) out[k] = add(carry, ex);
    carry = add(carry, tot);
  }
}

// The whole scan in one workgroup (small n): striped coalesced loads into
// LDS, all in flight together; each thread then sums a consecutive run, one
// workgroup scan places the runs, and each thread writes its run.
template <class T>
constexpr int64_t single_max() { return 32768 / (int64_t)sizeof(T); }  // 32 KiB of LDS

template <class T, class In>
__device__ inline T rec_any(const In *in, int64_t k) {
  if constexpr (std::is_same<T, U4>::value) return rec(in, k);
  else return in[k];
}

template <class T, class In = T>
__global__ __launch_bounds__(kBS) void k_scan_single(const In *__restrict__ in, T *__restrict__ out, int64_t n) {
  constexpr int64_t kMax = single_max<T>();
  __shared__ T buf[kMax];
  __shared__ T lds[kBS / kWave];
#pragma unroll
  for (int64_t i = 0; i < kMax / kBS; i++) {
    const int64_t k = i * kBS + threadIdx.x;
    if (k < n) buf[k] = rec_any<T>(in, k);
  }
  __syncthreads();
  constexpr int64_t per = kMax / kBS;
  const int64_t b0 = (int64_t)threadIdx.x * per, b1 = b0 + per < n ? b0 + per : n;
  T s = zero<T>();
  for (int64_t k = b0; k < b1; k++) s = add(s, buf[k]);
  T tot;
  T run = block_excl_scan(s, &tot, lds);
  for (int64_t k = b0; k < b1; k++) {
    out[k] = run;
    run = add(run, buf[k]);
  }
  if (threadIdx.x == 0) out[n] = tot;
}

template <class T>
void scan_impl(const T *in, T *out, int64_t n, T *tmp, hipStream_t s) {
  if (n <= single_max<T>()) {
    k_scan_single<T><<<dim3(1), dim3(kBS), 0, s>>>(in, out, n);
    return;
  }
  int64_t ntiles = ceil_div(n, kTile);
  k_scan_reduce<T><<<dim3((unsigned)ntiles), dim3(kBS), 0, s>>>(in, tmp, n);
  k_scan_part<T><<<dim3(1), dim3(kBS), 0, s>>>(tmp, ntiles, out + n);
  k_scan_down<T><<<dim3((unsigned)ntiles), dim3(kBS), 0, s>>>(in, out, tmp, n);
}

}  // namespace

int64_t scan_tmp_elems(int64_t n) { return ceil_div(n > 0 ? n : 1, kTile) + 1; }

template <class In>
static void scan_records(const In *in, U4 *out, int64_t n, U4 *tmp, hipStream_t s) {
  if (n <= single_max<U4>()) {
    k_scan_single<U4, In><<<dim3(1), dim3(kBS), 0, s>>>(in, out, n);
    return;
  }
  const int64_t ntiles = ceil_div(n, kTile);
  k_scan_reduce_u4<In><<<dim3((unsigned)ntiles), dim3(kBS), 0, s>>>(in, tmp, n);
  if (ntiles <= kFuseTiles) {
    k_scan_down_u4<In, true><<<dim3((unsigned)ntiles), dim3(kBS), 0, s>>>(in, out, tmp, n);
    return;
  }
  k_scan_part<U4><<<dim3(1), dim3(kBS), 0, s>>>(tmp, ntiles, out + n);
  k_scan_down_u4<In><<<dim3((unsigned)ntiles), dim3(kBS), 0, s>>>(in, out, tmp, n);
}

void scan_u4(const U4 *in, U4 *out, int64_t n, U4 *tmp, hipStream_t s) { scan_records<U4>(in, out, n, tmp, s); }
void scan_u4_packed(const uint32_t *in, U4 *out, int64_t n, U4 *tmp, hipStream_t s) {
  scan_records<uint32_t>(in, out, n, tmp, s);
}
void scan_u64(const uint64_t *in, uint64_t *out, int64_t n, uint64_t *tmp, hipStream_t s) {
  scan_impl<uint64_t>(in, out, n, tmp, s);
}

}  // namespace chr
