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

struct SecularTrap {
  double w[3];  // secular angular frequency per axis, (Omega/2) sqrt(a_k + q_k^2/2)
};

__device__ __forceinline__ void ion_secular(const SecularTrap& T, const double* x0,
                                            const double* v0, double t, double* x, double* v) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double w = T.w[k];
    if (w > 0.0) {
      double s, c;
      sincos(w * t, &s, &c);
      x[k] = x0[k] * c + v0[k] / w * s;
      v[k] = -x0[k] * w * s + v0[k] * c;
    } else {
      x[k] = x0[k] + v0[k] * t;
      v[k] = v0[k];
    }
  }
}

// Predicted duration of trajectory i of an ensemble (see schedule.h).
__device__ float predicted_duration(const double* __restrict__ y0, long long ld, long long i,
                                    float horizon, double r_exit, const SecularTrap& trap) {
  float d = horizon;
  if (r_exit > 0.0) {
    double xi[3], vi[3], xa[3], va[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      xi[k] = y0[k * ld + i];
      vi[k] = y0[(3 + k) * ld + i];
      xa[k] = y0[(6 + k) * ld + i];
      va[k] = y0[(9 + k) * ld + i];
    }
    const double R2 = r_exit * r_exit;
    // start: straight-line exit from the sphere of radius r_exit about the
    // trap centre (larger root of |x_a + v_a t| = r_exit), or 2 r / |v_a|
    const double vv = va[0] * va[0] + va[1] * va[1] + va[2] * va[2];
    const double xv = xa[0] * va[0] + xa[1] * va[1] + xa[2] * va[2];
    const double disc = xv * xv - vv * (xa[0] * xa[0] + xa[1] * xa[1] + xa[2] * xa[2] - R2);
    double t;
    if (disc > 0.0) {
      t = (sqrt(disc) - xv) / vv;
    } else {
      const double dx = xa[0] - xi[0], dy = xa[1] - xi[1], dz = xa[2] - xi[2];
      t = 2.0 * sqrt((dx * dx + dy * dy + dz * dz) / vv);
    }
    // refine: the ion follows its secular motion; Newton steps on
    // g(t) = |x_a + v_a t - x_ion(t)|^2 - r_exit^2, each kept only if it stays
    // within a factor 2 of the straight-line value.  A trajectory whose
    // duration is underestimated starts late and can end after everything
    // else, so a step that leaves that range (an overshoot, or a root on the
    // wrong side) is discarded.
    const double ts = t;
    for (int it = 0; it < 3; ++it) {
      if (!(t > 0.0) || !(t < (double)horizon)) break;
      double x[3], v[3];
      ion_secular(trap, xi, vi, t, x, v);
      double g = -R2, gp = 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double dk = xa[k] + va[k] * t - x[k];
        g += dk * dk;
        gp += 2.0 * dk * (va[k] - v[k]);
      }
      if (gp > 0.0) {
        const double tn = t - g / gp;
        if (tn > 0.5 * ts && tn < 2.0 * ts) t = tn;
      }
    }
    const float tf = (float)t;  // inf for an atom at rest; NaN sorts anywhere
    d = tf < horizon ? (tf > 0.0f ? tf : 0.0f) : horizon;
  }
  return d;
}

__global__ void ai_cost_key_kernel(const double* __restrict__ y0, long long n, long long ld,
                                   float horizon, double r_exit, SecularTrap trap,
                                   float* __restrict__ key, unsigned* __restrict__ idx) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  key[i] = predicted_duration(y0, ld, i, horizon, r_exit, trap);
  idx[i] = (unsigned)i;
}

// Global index j of a batch: its item by binary search over the items'
// offsets (increasing), then the item's prediction.
__global__ void ai_cost_key_batch_kernel(const ai_order_item* __restrict__ items, int count,
                                         long long total, float* __restrict__ key,
                                         unsigned* __restrict__ idx) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= total) return;
  int lo = 0, hi = count - 1;  // last item with offset <= j
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (items[mid].offset <= j)
      lo = mid;
    else
      hi = mid - 1;
  }
  const ai_order_item& it = items[lo];
  SecularTrap trap;
  for (int k = 0; k < 3; ++k) trap.w[k] = it.secular_omega[k];
  key[j] = predicted_duration(it.y0, it.ld, j - it.offset, (float)it.horizon, it.r_exit, trap);
  idx[j] = (unsigned)j;
}

constexpr size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

namespace {

// Workspace for n keys: the cost kernel's output, the sorted copy, and the
// radix sort's scratch; `launch` enqueues the cost kernel into key_in/idx_in.
template <class Launch>
hipError_t sort_by_key(int64_t n, unsigned** order, float** key, void** workspace,
                       hipStream_t stream, Launch launch) {
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
  launch(key_in, idx_in);
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

}  // namespace

hipError_t ai_longest_first_order(const double* y0, int64_t n, int64_t ld, double horizon,
                                  double r_exit, const double secular_omega[3],
                                  unsigned** order, float** key,
                                  void** workspace, hipStream_t stream) {
  SecularTrap trap;
  for (int k = 0; k < 3; ++k) trap.w[k] = secular_omega[k];
  const unsigned threads = 256;
  const unsigned blocks = (unsigned)((n + threads - 1) / threads);
  return sort_by_key(n, order, key, workspace, stream, [&](float* key_in, unsigned* idx_in) {
    hipLaunchKernelGGL(ai_cost_key_kernel, dim3(blocks), dim3(threads), 0, stream, y0,
                       (long long)n, (long long)ld, (float)horizon, r_exit, trap, key_in,
                       idx_in);
  });
}

hipError_t ai_longest_first_order_batch(const ai_order_item* items, int count, int64_t total,
                                        unsigned** order, float** key, void** workspace,
                                        hipStream_t stream) {
  if (count <= 0) return hipErrorInvalidValue;
  const unsigned threads = 256;
  const unsigned blocks = (unsigned)((total + threads - 1) / threads);
  return sort_by_key(total, order, key, workspace, stream, [&](float* key_in, unsigned* idx_in) {
    hipLaunchKernelGGL(ai_cost_key_batch_kernel, dim3(blocks), dim3(threads), 0, stream, items,
                       count, (long long)total, key_in, idx_in);
  });
}
