// schedule.hip -- longest-predicted-first ordering of an ensemble (see
// schedule.h).  Trajectory costs differ by more than an order of magnitude
// (slow atoms take up to the full integration span), and a long trajectory
// started late keeps its wave alive after every other wave has drained.
// Starting the longest first lets the shorter ones fill in around them; the
// order only decides which lane integrates which trajectory, so results do
// not depend on it.
#include "schedule.h"

#include <cmath>
#include <cstring>
#include <mutex>

namespace {

// The ion on its secular orbit: per axis a harmonic oscillation at the
// secular frequency w (free flight where w = 0) from (x0, v0) at t0.
__device__ __forceinline__ void ion_secular(const ai_order_model& M, const double* x0,
                                            const double* v0, double t, double* x, double* v) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double w = M.secular_omega[k];
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

// The span a close pass adds to a trajectory that exits at t (see
// AI_ORDER_CLOSE_* in schedule.h): the closest approach of the atom's
// straight line to the ion's secular orbit before t, by Newton steps on
// d/dt |d|^2 = 0 from the closest approach of the initial relative motion,
// kept within [0, t].  Single precision: the radii that matter are hundreds to
// thousands of a0, positions at most ~1e6 a0.
__device__ float close_pass_span(const double* xi_d, const double* vi_d, const double* xa_d,
                                 const double* va_d, const ai_order_model& M, double t_d) {
  if (!(M.close_span > 0.0f) || !(t_d > 0.0)) return 0.0f;
  const float t = (float)t_d;
  float xi[3], vi[3], xa[3], va[3], w[3];
  float d0v = 0.0f, uu = 0.0f;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    xi[k] = (float)xi_d[k];
    vi[k] = (float)vi_d[k];
    xa[k] = (float)xa_d[k];
    va[k] = (float)va_d[k];
    w[k] = (float)M.secular_omega[k];
    const float u = va[k] - vi[k];
    d0v += (xa[k] - xi[k]) * u;
    uu += u * u;
  }
  float tc = uu > 0.0f ? fminf(fmaxf(-d0v / uu, 0.0f), t) : 0.0f;
  float r2c = 0.0f;
  for (int it = 0; it < 4; ++it) {
    float f1 = 0.0f, f2 = 0.0f;
    r2c = 0.0f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      float x, v;
      if (w[k] > 0.0f) {
        float sn, cs;
        sincosf(w[k] * tc, &sn, &cs);
        x = xi[k] * cs + vi[k] / w[k] * sn;
        v = vi[k] * cs - xi[k] * w[k] * sn;
      } else {
        x = xi[k] + vi[k] * tc;
        v = vi[k];
      }
      const float dk = xa[k] + va[k] * tc - x, uk = va[k] - v;
      r2c += dk * dk;
      f1 += dk * uk;
      f2 += uk * uk + dk * w[k] * w[k] * x;
    }
    if (f2 > 0.0f) tc = fminf(fmaxf(tc - f1 / f2, 0.0f), t);
  }
  const float frac = (float)((AI_ORDER_CLOSE_R_OUT - (double)sqrtf(r2c)) /
                             (AI_ORDER_CLOSE_R_OUT - AI_ORDER_CLOSE_R_IN));
  return M.close_span * fminf(fmaxf(frac, 0.0f), 1.0f);
}

// Analytic duration (see schedule.h): the straight-line exit of the atom from
// the sphere of radius r_exit about the trap centre, refined by Newton steps
// against the ion's secular orbit.
__device__ float analytic_duration(const double* __restrict__ y0, long long ld, long long i,
                                   const ai_order_model& M) {
  const float horizon = M.horizon;
  double xi[3], vi[3], xa[3], va[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    xi[k] = y0[k * ld + i];
    vi[k] = y0[(3 + k) * ld + i];
    xa[k] = y0[(6 + k) * ld + i];
    va[k] = y0[(9 + k) * ld + i];
  }
  const double R2 = M.r_exit * M.r_exit;
  // start: the larger root of |x_a + v_a t| = r_exit, or 2 r / |v_a|
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
  // refine on g(t) = |x_a + v_a t - x_ion(t)|^2 - r_exit^2, keeping a step
  // only within a factor 2 of the straight-line value: an underestimated
  // trajectory starts late and can end after everything else, so a step that
  // leaves that range (an overshoot, or a root on the wrong side) is dropped
  const double ts = t;
  for (int it = 0; it < 3; ++it) {
    if (!(t > 0.0) || !(t < (double)horizon)) break;
    double x[3], v[3];
    ion_secular(M, xi, vi, t, x, v);
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
  const float close = close_pass_span(xi, vi, xa, va, M, t);
  const float tf = (float)t + close;  // inf for an atom at rest; NaN sorts anywhere
  return tf < horizon ? (tf > 0.0f ? tf : 0.0f) : horizon;
}

// Sampled duration (see schedule.h): the exit rule on samples of the exact
// linear trap motion.
__device__ float sampled_duration(const double* __restrict__ y0, long long ld, long long i,
                                  const ai_order_model& M) {
  const float horizon = M.horizon;
  double xi[3], vi[3], xa[3], va[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    xi[k] = y0[k * ld + i];
    vi[k] = y0[(3 + k) * ld + i];
    xa[k] = y0[(6 + k) * ld + i];
    va[k] = y0[(9 + k) * ld + i];
  }
  // t0: a pair that is not closing in counts as past its closest approach
  double dot = 0.0, r2_0 = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double rel = xi[k] - xa[k];
    dot += rel * (vi[k] - va[k]);
    r2_0 += rel * rel;
  }
  float s0[3], s1[3], pa[3], wa[3];  // ion (x, v) at the current period's start; atom
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    s0[k] = (float)xi[k];
    s1[k] = (float)vi[k];
    pa[k] = (float)xa[k];
    wa[k] = (float)va[k];
  }
  bool approached = dot >= 0.0;
  bool falling = dot < 0.0;
  float prev = (float)r2_0;
  const float far2 = 1e4f * M.r_exit2;  // the ion has left the trap (unstable axis)
  float t_exit = -1.0f;
  for (int P = 0; P < M.periods; ++P) {
    const float base = (float)(P * AI_ORDER_SAMPLES);
    float hit = -1.0f;
#pragma unroll
    for (int j = 0; j < AI_ORDER_SAMPLES; ++j) {
      const float t = (base + (float)(j + 1)) * M.dt;
      float r2 = 0.0f;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float x = fmaf(M.phi[k][j][0], s0[k], M.phi[k][j][1] * s1[k]);
        const float dk = x - fmaf(wa[k], t, pa[k]);
        r2 = fmaf(dk, dk, r2);
      }
      // a local minimum of the distance between two samples is a closest approach
      const bool rising = r2 >= prev;
      approached = approached || (falling && rising);
      falling = !rising;
      prev = r2;
      if (hit < 0.0f && ((approached && r2 > M.r_exit2) || !(r2 < far2))) hit = t;
    }
    if (hit >= 0.0f) {
      t_exit = hit;
      break;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float x = fmaf(M.mono[k][0], s0[k], M.mono[k][1] * s1[k]);
      const float v = fmaf(M.mono[k][2], s0[k], M.mono[k][3] * s1[k]);
      s0[k] = x;
      s1[k] = v;
    }
  }
  if (t_exit < 0.0f) {
    // still inside after the searched span: the straight-line exit from the
    // sphere of radius r_exit about the ion's start, but not before the span's end
    const float span = (float)(M.periods * AI_ORDER_SAMPLES) * M.dt;
    double vv = 0.0, xv = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      vv += va[k] * va[k];
      xv += (xa[k] - xi[k]) * va[k];
    }
    const double disc = xv * xv - vv * (r2_0 - (double)M.r_exit2);
    const float line = disc > 0.0 && vv > 0.0 ? (float)((sqrt(disc) - xv) / vv) : horizon;
    t_exit = fmaxf(span, line);
  }
  t_exit += close_pass_span(xi, vi, xa, va, M, (double)t_exit);
  return t_exit < horizon ? t_exit : horizon;  // NaN sorts anywhere
}

// Predicted cost of trajectory i of an ensemble (see schedule.h).
__device__ float predicted_cost(const double* __restrict__ y0, long long ld, long long i,
                                const ai_order_model& M) {
  if (!(M.r_exit > 0.0)) return M.horizon * M.rate;
  return (M.sampled ? sampled_duration(y0, ld, i, M) : analytic_duration(y0, ld, i, M)) * M.rate;
}

// The sort key: the cost on AI_ORDER_CODES levels from 0 to the largest
// possible cost (a non-finite prediction, from a non-finite initial state,
// takes the lowest).
__device__ __forceinline__ unsigned cost_code(float cost, float scale) {
  const float c = cost * scale;
  return c > 0.0f ? (unsigned)fminf(c, (float)(AI_ORDER_CODES - 1)) : 0u;
}

__global__ void ai_cost_key_kernel(const double* __restrict__ y0, long long n, long long ld,
                                   ai_order_model model, float scale,
                                   unsigned* __restrict__ key, unsigned* __restrict__ idx) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  key[i] = cost_code(predicted_cost(y0, ld, i, model), scale);
  idx[i] = (unsigned)i;
}

// Global index j of a batch: its item by binary search over the items'
// offsets (increasing), then the item's prediction.
__global__ void ai_cost_key_batch_kernel(const ai_order_item* __restrict__ items, int count,
                                         long long total, float scale,
                                         unsigned* __restrict__ key, unsigned* __restrict__ idx) {
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
  key[j] = cost_code(predicted_cost(it.y0, it.ld, j - it.offset, it.model), scale);
  idx[j] = (unsigned)j;
}

constexpr size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

namespace {

// ---- Counting sort of the cost codes, descending ----
//
// The codes have AI_ORDER_CODE_BITS bits, so one counting pass orders them:
// the keys are cut into tiles (one block each); a first kernel counts each
// tile's codes in LDS; an exclusive scan over the counts, taken code by code
// from the largest and tile by tile within a code, gives every (code, tile)
// pair its first output position; a scatter kernel hands out positions within
// a pair by LDS atomics.  Equal codes therefore come out in no fixed order,
// which changes nothing but which lane integrates which trajectory.  Every
// word of the workspace that is read is written first by these kernels, so
// the sort needs no memset (and a stream capture records kernels only).
constexpr int SORT_THREADS = 256;
constexpr int SORT_MAX_TILES = 1024;  // counts stay at most 16 MiB
constexpr int SORT_ROW_THREADS = 256;
constexpr int SORT_BASE_THREADS = 1024;
static_assert(AI_ORDER_CODES % SORT_BASE_THREADS == 0, "rows per thread of the base scan");
static_assert(SORT_MAX_TILES % SORT_ROW_THREADS == 0, "tiles per thread of the row scan");

struct SortLayout {
  int tiles;     // blocks of the count and scatter kernels
  int64_t tile;  // keys per tile, a multiple of SORT_THREADS
};

SortLayout sort_layout(int64_t n) {
  int64_t tiles = (n + 4095) / 4096;
  tiles = tiles < 1 ? 1 : (tiles > SORT_MAX_TILES ? SORT_MAX_TILES : tiles);
  int64_t tile = (n + tiles - 1) / tiles;
  tile = (tile + SORT_THREADS - 1) / SORT_THREADS * SORT_THREADS;
  SortLayout L;
  L.tile = tile;
  L.tiles = (int)((n + tile - 1) / tile);
  return L;
}

// Row r of the counts holds code AI_ORDER_CODES - 1 - r, so that rows in
// increasing order are codes in decreasing order.
__device__ __forceinline__ unsigned code_row(unsigned key) {
  return AI_ORDER_CODES - 1u - (key < AI_ORDER_CODES ? key : AI_ORDER_CODES - 1u);
}

// counts[r * tiles + t]: keys of tile t in row r.
__global__ __launch_bounds__(SORT_THREADS) void ai_sort_count_kernel(
    const unsigned* __restrict__ key, long long n, long long tile, int tiles,
    unsigned* __restrict__ counts) {
  __shared__ unsigned h[AI_ORDER_CODES];
  for (int r = threadIdx.x; r < (int)AI_ORDER_CODES; r += SORT_THREADS) h[r] = 0u;
  __syncthreads();
  const long long begin = (long long)blockIdx.x * tile;
  const long long end = begin + tile < n ? begin + tile : n;
  for (long long i = begin + threadIdx.x; i < end; i += SORT_THREADS)
    atomicAdd(&h[code_row(key[i])], 1u);
  __syncthreads();
  for (int r = threadIdx.x; r < (int)AI_ORDER_CODES; r += SORT_THREADS)
    counts[(long long)r * tiles + blockIdx.x] = h[r];
}

// Inclusive scan of one value per thread over a block of THREADS threads
// (Hillis-Steele in LDS); `total` receives the block's sum.
template <int THREADS>
__device__ __forceinline__ unsigned block_inclusive_scan(unsigned v, unsigned* lds,
                                                         unsigned& total) {
  lds[threadIdx.x] = v;
  __syncthreads();
  for (int d = 1; d < THREADS; d <<= 1) {
    const unsigned add = threadIdx.x >= (unsigned)d ? lds[threadIdx.x - d] : 0u;
    __syncthreads();
    lds[threadIdx.x] += add;
    __syncthreads();
  }
  const unsigned r = lds[threadIdx.x];
  total = lds[THREADS - 1];
  __syncthreads();
  return r;
}

// One block per row: the row's counts become offsets within the row
// (exclusive scan over the tiles); row_total[r] receives the row's sum.
__global__ __launch_bounds__(SORT_ROW_THREADS) void ai_sort_row_kernel(
    unsigned* __restrict__ counts, int tiles, unsigned* __restrict__ row_total) {
  __shared__ unsigned lds[SORT_ROW_THREADS];
  unsigned* row = counts + (long long)blockIdx.x * tiles;
  const int per = (tiles + SORT_ROW_THREADS - 1) / SORT_ROW_THREADS;  // at most 4
  const int first = threadIdx.x * per;
  unsigned local[SORT_MAX_TILES / SORT_ROW_THREADS];
  unsigned sum = 0u;
#pragma unroll
  for (int j = 0; j < SORT_MAX_TILES / SORT_ROW_THREADS; ++j) {
    const int t = first + j;
    local[j] = (j < per && t < tiles) ? row[t] : 0u;
    sum += local[j];
  }
  unsigned total = 0u;
  unsigned run = block_inclusive_scan<SORT_ROW_THREADS>(sum, lds, total) - sum;
#pragma unroll
  for (int j = 0; j < SORT_MAX_TILES / SORT_ROW_THREADS; ++j) {
    const int t = first + j;
    if (j < per && t < tiles) row[t] = run;
    run += local[j];
  }
  if (threadIdx.x == 0) row_total[blockIdx.x] = total;
}

// One block: row_base[r] = the sum of the rows before r.
__global__ __launch_bounds__(SORT_BASE_THREADS) void ai_sort_base_kernel(
    const unsigned* __restrict__ row_total, unsigned* __restrict__ row_base) {
  __shared__ unsigned lds[SORT_BASE_THREADS];
  constexpr int PER = AI_ORDER_CODES / SORT_BASE_THREADS;
  unsigned local[PER];
  unsigned sum = 0u;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    local[j] = row_total[threadIdx.x * PER + j];
    sum += local[j];
  }
  unsigned total = 0u;
  unsigned run = block_inclusive_scan<SORT_BASE_THREADS>(sum, lds, total) - sum;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    row_base[threadIdx.x * PER + j] = run;
    run += local[j];
  }
}

// Every key of tile t to its position: its row's base, the tile's offset in
// the row, and a rank among the tile's keys of that row.
__global__ __launch_bounds__(SORT_THREADS) void ai_sort_scatter_kernel(
    const unsigned* __restrict__ key_in, const unsigned* __restrict__ idx_in, long long n,
    long long tile, int tiles, const unsigned* __restrict__ offsets,
    const unsigned* __restrict__ row_base, unsigned* __restrict__ key_out,
    unsigned* __restrict__ idx_out) {
  __shared__ unsigned cursor[AI_ORDER_CODES];
  for (int r = threadIdx.x; r < (int)AI_ORDER_CODES; r += SORT_THREADS)
    cursor[r] = row_base[r] + offsets[(long long)r * tiles + blockIdx.x];
  __syncthreads();
  const long long begin = (long long)blockIdx.x * tile;
  const long long end = begin + tile < n ? begin + tile : n;
  for (long long i = begin + threadIdx.x; i < end; i += SORT_THREADS) {
    const unsigned k = key_in[i];
    const unsigned pos = atomicAdd(&cursor[code_row(k)], 1u);
    key_out[pos] = k;
    idx_out[pos] = idx_in[i];
  }
}

// Workspace for n keys: the cost kernel's output, the sorted copy, and the
// counting sort's counts and row sums.
size_t workspace_bytes(int64_t n) {
  const SortLayout L = sort_layout(n);
  return 4 * align256(sizeof(unsigned) * (size_t)n) +
         align256(sizeof(unsigned) * (size_t)AI_ORDER_CODES * (size_t)L.tiles) +
         2 * align256(sizeof(unsigned) * (size_t)AI_ORDER_CODES);
}

// ext: a caller's workspace of ext_bytes (nothing is allocated, *workspace
// stays NULL), or NULL to allocate one on the stream.
template <class Launch>
hipError_t sort_by_key(int64_t n, unsigned** order, unsigned** key, void** workspace,
                       hipStream_t stream, Launch launch, char* ext = nullptr,
                       size_t ext_bytes = 0) {
  *order = nullptr;
  *key = nullptr;
  *workspace = nullptr;
  if (n <= 0 || n > 0xffffffffLL) return hipErrorInvalidValue;
  const SortLayout L = sort_layout(n);
  const size_t total = workspace_bytes(n);
  const size_t ubytes = align256(sizeof(unsigned) * (size_t)n);
  const size_t cbytes = align256(sizeof(unsigned) * (size_t)AI_ORDER_CODES * (size_t)L.tiles);
  const size_t rbytes = align256(sizeof(unsigned) * (size_t)AI_ORDER_CODES);
  hipError_t e = hipSuccess;
  char* base = ext;
  if (ext) {
    if (total > ext_bytes) return hipErrorInvalidValue;
  } else if ((e = hipMallocAsync((void**)&base, total, stream)) != hipSuccess) {
    return e;
  }
  unsigned* key_in = (unsigned*)base;
  unsigned* key_out = (unsigned*)(base + ubytes);
  unsigned* idx_in = (unsigned*)(base + 2 * ubytes);
  unsigned* idx_out = (unsigned*)(base + 3 * ubytes);
  unsigned* counts = (unsigned*)(base + 4 * ubytes);
  unsigned* row_total = (unsigned*)(base + 4 * ubytes + cbytes);
  unsigned* row_base = (unsigned*)(base + 4 * ubytes + cbytes + rbytes);
  launch(key_in, idx_in);
  if ((e = hipGetLastError()) == hipSuccess) {
    hipLaunchKernelGGL(ai_sort_count_kernel, dim3(L.tiles), dim3(SORT_THREADS), 0, stream,
                       key_in, (long long)n, (long long)L.tile, L.tiles, counts);
    hipLaunchKernelGGL(ai_sort_row_kernel, dim3(AI_ORDER_CODES), dim3(SORT_ROW_THREADS), 0,
                       stream, counts, L.tiles, row_total);
    hipLaunchKernelGGL(ai_sort_base_kernel, dim3(1), dim3(SORT_BASE_THREADS), 0, stream,
                       row_total, row_base);
    hipLaunchKernelGGL(ai_sort_scatter_kernel, dim3(L.tiles), dim3(SORT_THREADS), 0, stream,
                       key_in, idx_in, (long long)n, (long long)L.tile, L.tiles, counts,
                       row_base, key_out, idx_out);
    e = hipGetLastError();
  }
  if (e != hipSuccess) {
    if (!ext) (void)hipFreeAsync(base, stream);
    return e;
  }
  *order = idx_out;
  *key = key_out;
  *workspace = ext ? nullptr : base;
  return hipSuccess;
}

// Scale from costs to codes for costs up to cost_max.
float code_scale(double cost_max) {
  return cost_max > 0.0 && std::isfinite(cost_max) ? (float)(AI_ORDER_CODES / cost_max) : 0.0f;
}

}  // namespace

namespace {

// The per-axis matrices of ai_order_model, which depend on the trap alone.
struct TrapTables {
  double a[3], q[3], omega_rf, t0;
  float phi[3][AI_ORDER_SAMPLES][2];
  float mono[3][4];
};

// Fundamental solutions of x'' = -(a_k + 2 q_k cos(omega_rf t)) omega_rf^2 / 4 x
// from t0 over one period, classical RK4 with SUB steps per sample; the trap's
// cosine on the half-step grid is shared by all axes.
void trap_tables(TrapTables& T, double period) {
  constexpr int SUB = 32;
  constexpr int STEPS = AI_ORDER_SAMPLES * SUB;
  const double h = period / STEPS;
  double cosine[2 * STEPS + 1];
  for (int i = 0; i <= 2 * STEPS; ++i) cosine[i] = std::cos(T.omega_rf * (T.t0 + 0.5 * h * i));
  const double c = 0.25 * T.omega_rf * T.omega_rf;
  for (int k = 0; k < 3; ++k) {
    if (k > 0 && T.a[k] == T.a[k - 1] && T.q[k] == T.q[k - 1]) {  // the previous axis's equation
      for (int j = 0; j < AI_ORDER_SAMPLES; ++j)
        for (int col = 0; col < 2; ++col) T.phi[k][j][col] = T.phi[k - 1][j][col];
      for (int e = 0; e < 4; ++e) T.mono[k][e] = T.mono[k - 1][e];
      continue;
    }
    auto acc = [&](int half_steps, double x) {
      return -(T.a[k] + 2.0 * T.q[k] * cosine[half_steps]) * c * x;
    };
    for (int col = 0; col < 2; ++col) {
      double x = col == 0 ? 1.0 : 0.0, v = col == 0 ? 0.0 : 1.0;
      for (int i = 0; i < STEPS; ++i) {
        const double k1x = v, k1v = acc(2 * i, x);
        const double k2x = v + 0.5 * h * k1v, k2v = acc(2 * i + 1, x + 0.5 * h * k1x);
        const double k3x = v + 0.5 * h * k2v, k3v = acc(2 * i + 1, x + 0.5 * h * k2x);
        const double k4x = v + h * k3v, k4v = acc(2 * i + 2, x + h * k3x);
        x += h / 6.0 * (k1x + 2.0 * k2x + 2.0 * k3x + k4x);
        v += h / 6.0 * (k1v + 2.0 * k2v + 2.0 * k3v + k4v);
        if ((i + 1) % SUB == 0) T.phi[k][(i + 1) / SUB - 1][col] = (float)x;
      }
      T.mono[k][col] = (float)x;      // x row
      T.mono[k][2 + col] = (float)v;  // v row
    }
  }
}

// Recently built tables (a batch repeats traps; a serving loop repeats calls).
constexpr int TABLE_CACHE = 16;
std::mutex table_mutex;
TrapTables table_cache[TABLE_CACHE];
int table_count = 0, table_next = 0;

bool same_trap(const TrapTables& T, const double a[3], const double q[3], double omega_rf,
               double t0) {
  for (int k = 0; k < 3; ++k)
    if (T.a[k] != a[k] || T.q[k] != q[k]) return false;
  return T.omega_rf == omega_rf && T.t0 == t0;
}

}  // namespace

ai_order_model ai_make_order_model(const double a[3], const double q[3], double omega_rf,
                                   double r_exit, double t0, double tmax, double rtol,
                                   bool sampled) {
  ai_order_model m{};
  m.sampled = sampled ? 1 : 0;
  m.r_exit = r_exit;
  for (int k = 0; k < 3; ++k)
    m.secular_omega[k] = 0.5 * std::fabs(omega_rf) * std::sqrt(std::fmax(a[k] + 0.5 * q[k] * q[k], 0.0));
  const double horizon = tmax - t0;
  const double w = std::fabs(omega_rf);
  // one RF period (any interval for a static trap, whose equation is autonomous)
  const double period = w > 0.0 ? 6.283185307179586 / w : horizon / AI_ORDER_MAX_PERIODS;
  m.horizon = (float)horizon;
  m.close_span = w > 0.0 ? (float)(AI_ORDER_CLOSE_PERIODS * period) : 0.0f;
  m.r_exit2 = (float)(r_exit * r_exit * (1.0 + 0x1p-12));
  m.dt = (float)(period / AI_ORDER_SAMPLES);
  m.periods = (int)std::fmin(std::ceil(horizon / period), (double)AI_ORDER_MAX_PERIODS);
  double qmax = 0.0;
  for (int k = 0; k < 3; ++k) qmax = std::fmax(qmax, std::fabs(q[k]));
  // ode45's attempts per unit time grow with the RF frequency, slowly with q
  // (exponent fitted to measured attempt counts) and as rtol^(-1/5)
  m.rate = (float)((w > 0.0 ? w : 1.0 / horizon) * std::pow(std::fmax(qmax, 1e-3), 0.3) *
                   std::pow(rtol, -0.2));

  if (!sampled) return m;
  TrapTables T;
  bool found = false;
  {
    std::lock_guard<std::mutex> lock(table_mutex);
    for (int i = 0; i < table_count && !found; ++i)
      if (same_trap(table_cache[i], a, q, omega_rf, t0)) {
        T = table_cache[i];
        found = true;
      }
  }
  if (!found) {
    for (int k = 0; k < 3; ++k) {
      T.a[k] = a[k];
      T.q[k] = q[k];
    }
    T.omega_rf = omega_rf;
    T.t0 = t0;
    // the static trap's interval depends on the horizon: not cached
    trap_tables(T, period);
    if (w > 0.0) {
      std::lock_guard<std::mutex> lock(table_mutex);
      table_cache[table_next] = T;
      table_next = (table_next + 1) % TABLE_CACHE;
      if (table_count < TABLE_CACHE) ++table_count;
    }
  }
  std::memcpy(m.phi, T.phi, sizeof m.phi);
  std::memcpy(m.mono, T.mono, sizeof m.mono);
  return m;
}

size_t ai_order_workspace_bytes(int64_t n, hipStream_t) {
  return n > 0 && n <= 0xffffffffLL ? workspace_bytes(n) : 0;
}

hipError_t ai_longest_first_order(const double* y0, int64_t n, int64_t ld,
                                  const ai_order_model& model, unsigned** order, unsigned** key,
                                  void** workspace, hipStream_t stream, void* ext,
                                  size_t ext_bytes) {
  const float scale = code_scale((double)model.horizon * model.rate);
  const unsigned threads = 256;
  const unsigned blocks = (unsigned)((n + threads - 1) / threads);
  return sort_by_key(
      n, order, key, workspace, stream,
      [&](unsigned* key_in, unsigned* idx_in) {
        hipLaunchKernelGGL(ai_cost_key_kernel, dim3(blocks), dim3(threads), 0, stream, y0,
                           (long long)n, (long long)ld, model, scale, key_in, idx_in);
      },
      (char*)ext, ext_bytes);
}

hipError_t ai_longest_first_order_batch(const ai_order_item* items, int count, int64_t total,
                                        double cost_max, unsigned** order, unsigned** key,
                                        void** workspace, hipStream_t stream) {
  const float scale = code_scale(cost_max);
  if (count <= 0) return hipErrorInvalidValue;
  const unsigned threads = 256;
  const unsigned blocks = (unsigned)((total + threads - 1) / threads);
  return sort_by_key(total, order, key, workspace, stream, [&](unsigned* key_in, unsigned* idx_in) {
    hipLaunchKernelGGL(ai_cost_key_batch_kernel, dim3(blocks), dim3(threads), 0, stream, items,
                       count, (long long)total, scale, key_in, idx_in);
  });
}
