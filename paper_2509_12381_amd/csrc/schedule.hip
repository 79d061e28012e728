// schedule.hip -- longest-predicted-first ordering of an ensemble (see
// schedule.h).  Trajectory costs differ by more than an order of magnitude
// (slow atoms take up to the full integration span), and a long trajectory
// started late keeps its wave alive after every other wave has drained.
// Starting the longest first lets the shorter ones fill in around them; the
// order only decides which lane integrates which trajectory, so results do
// not depend on it.
#include "schedule.h"

#include <rocprim/device/device_radix_sort.hpp>

namespace {

__global__ void ai_cost_key_kernel(const double* __restrict__ y0, long long n, long long ld,
                                   float horizon, double r_exit, float* __restrict__ key,
                                   unsigned* __restrict__ idx) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float d = horizon;
  if (r_exit > 0.0) {
    // the ion stays near the trap centre: straight-line exit of the atom from
    // the sphere of radius r_exit about the origin, larger root of
    // |x + v t| = r_exit; 2 |x_atom - x_ion| / |v| if the line misses it
    const double x = y0[6 * ld + i], y = y0[7 * ld + i], z = y0[8 * ld + i];
    const double vx = y0[9 * ld + i], vy = y0[10 * ld + i], vz = y0[11 * ld + i];
    const double vv = vx * vx + vy * vy + vz * vz;
    const double xv = x * vx + y * vy + z * vz;
    const double disc = xv * xv - vv * (x * x + y * y + z * z - r_exit * r_exit);
    double t;
    if (disc > 0.0) {
      t = (sqrt(disc) - xv) / vv;
    } else {
      const double dx = x - y0[i], dy = y - y0[ld + i], dz = z - y0[2 * ld + i];
      t = 2.0 * sqrt((dx * dx + dy * dy + dz * dz) / vv);
    }
    const float tf = (float)t;  // inf for an atom at rest; NaN sorts anywhere
    d = tf < horizon ? (tf > 0.0f ? tf : 0.0f) : horizon;
  }
  key[i] = d;
  idx[i] = (unsigned)i;
}

constexpr size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

hipError_t ai_longest_first_order(const double* y0, int64_t n, int64_t ld, double horizon,
                                  double r_exit, unsigned** order, float** key,
                                  void** workspace, hipStream_t stream) {
  *order = nullptr;
  *key = nullptr;
  *workspace = nullptr;
  if (n <= 0 || n > 0xffffffffLL) return hipErrorInvalidValue;
  const unsigned size = (unsigned)n;
  size_t temp_bytes = 0;
  hipError_t e = rocprim::radix_sort_pairs_desc(nullptr, temp_bytes, (float*)nullptr,
                                                (float*)nullptr, (unsigned*)nullptr,
                                                (unsigned*)nullptr, size, 0, 32, stream);
  if (e != hipSuccess) return e;
  const size_t fbytes = align256(sizeof(float) * (size_t)n);
  const size_t ubytes = align256(sizeof(unsigned) * (size_t)n);
  const size_t total = 2 * fbytes + 2 * ubytes + align256(temp_bytes);
  char* base = nullptr;
  if ((e = hipMallocAsync((void**)&base, total, stream)) != hipSuccess) return e;
  float* key_in = (float*)base;
  float* key_out = (float*)(base + fbytes);
  unsigned* idx_in = (unsigned*)(base + 2 * fbytes);
  unsigned* idx_out = (unsigned*)(base + 2 * fbytes + ubytes);
  void* temp = base + 2 * fbytes + 2 * ubytes;
  const unsigned threads = 256;
  const unsigned blocks = (unsigned)((n + threads - 1) / threads);
  hipLaunchKernelGGL(ai_cost_key_kernel, dim3(blocks), dim3(threads), 0, stream, y0,
                     (long long)n, (long long)ld, (float)horizon, r_exit, key_in, idx_in);
  if ((e = hipGetLastError()) == hipSuccess)
    e = rocprim::radix_sort_pairs_desc(temp, temp_bytes, key_in, key_out, idx_in, idx_out, size,
                                       0, 32, stream);
  if (e != hipSuccess) {
    (void)hipFreeAsync(base, stream);
    return e;
  }
  *order = idx_out;
  *key = key_out;
  *workspace = base;
  return hipSuccess;
}
