// scan.hip -- device-wide exclusive prefix sums for gfx950.
//
// Three launches: per-tile totals (coalesced striped loads), one workgroup
// scanning the tile totals, and a downsweep that scans each tile as eight
// 256-element rows with wave-level shuffles and adds the tile's prefix.
// Small inputs take one launch.
#include "scan.h"

#include "chr_device.h"

namespace chr {
namespace {

constexpr int kBS = 256;
constexpr int kIPT = 8;
constexpr int kTile = kBS * kIPT;

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

template <class T>
__global__ __launch_bounds__(kBS) void k_scan_single(const T *__restrict__ in, T *__restrict__ out, int64_t n) {
  constexpr int64_t kMax = single_max<T>();
  __shared__ T buf[kMax];
  __shared__ T lds[kBS / kWave];
#pragma unroll
  for (int64_t i = 0; i < kMax / kBS; i++) {
    const int64_t k = i * kBS + threadIdx.x;
    if (k < n) buf[k] = in[k];
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

void scan_u4(const U4 *in, U4 *out, int64_t n, U4 *tmp, hipStream_t s) { scan_impl<U4>(in, out, n, tmp, s); }
void scan_u64(const uint64_t *in, uint64_t *out, int64_t n, uint64_t *tmp, hipStream_t s) {
  scan_impl<uint64_t>(in, out, n, tmp, s);
}

}  // namespace chr
