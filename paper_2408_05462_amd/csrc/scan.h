// scan.h -- device-wide exclusive prefix sums (reduce, scan partials, downsweep).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace chr {

struct U4 {
  uint32_t x, y, z, w;
};

// Scratch elements (of the scanned type) needed to scan n elements.
int64_t scan_tmp_elems(int64_t n);

// out[i] = in[0] + ... + in[i-1] for i in [0, n]; out must hold n+1 elements
// (out[n] is the total).  tmp holds scan_tmp_elems(n) elements.
void scan_u4(const U4 *in, U4 *out, int64_t n, U4 *tmp, hipStream_t s);
// The same over marching cubes' word counts stored as 32-bit records:
// vertices in bits 0-7 (at most 192), triangles in bits 8-16 (at most 320),
// crossing points in bits 17-23 and active cells in bits 24-30 (at most 64).
void scan_u4_packed(const uint32_t *in, U4 *out, int64_t n, U4 *tmp, hipStream_t s);
void scan_u64(const uint64_t *in, uint64_t *out, int64_t n, uint64_t *tmp, hipStream_t s);

}  // namespace chr
