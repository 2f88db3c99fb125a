// Rows of the heuristic first-sweep set.  The paper (Sec. 6) names a
// heuristic a-priori subset of the rows for the first sweep without fixing a
// rule; the library's reading marks the rows a step carries from the
// previous one and the rows a stimulus overwrites, then grows the marks by
// mesh neighbours (the pattern of A: vertices that share a simplex).  The
// selection kernels compact rows whose mark is 1.
#include "kernels.hpp"

namespace sdc {

namespace {

constexpr int kMarkBlock = 256;

__global__ __launch_bounds__(kMarkBlock) void k_mark_clear(double* __restrict__ mark, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kMarkBlock + threadIdx.x;
  if (i < n) mark[i] = 0.0;
}

__global__ __launch_bounds__(kMarkBlock) void k_mark_rows(const int32_t* __restrict__ rows, int64_t n,
                                                          double* __restrict__ mark) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * kMarkBlock + threadIdx.x;
  if (q < n) mark[rows[q]] = 1.0;
}

// One ring: out_i = max(in_j) over the row's pattern (which holds i itself).
__global__ __launch_bounds__(kMarkBlock) void k_mark_grow(const int32_t* __restrict__ rowptr,
                                                          const int32_t* __restrict__ col,
                                                          const double* __restrict__ in,
                                                          double* __restrict__ out, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kMarkBlock + threadIdx.x;
  if (i >= n) return;
  double m = 0.0;
  for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) m = fmax(m, in[col[e]]);
  out[i] = m;
}

inline unsigned grid_of(int64_t n) { return static_cast<unsigned>((n + kMarkBlock - 1) / kMarkBlock); }

}  // namespace

void launch_mark_clear(hipStream_t s, double* mark, int64_t n) {
  if (n > 0) k_mark_clear<<<grid_of(n), kMarkBlock, 0, s>>>(mark, n);
}

void launch_mark_rows(hipStream_t s, const int32_t* rows, int64_t n, double* mark) {
  if (n > 0) k_mark_rows<<<grid_of(n), kMarkBlock, 0, s>>>(rows, n, mark);
}

void launch_mark_grow(hipStream_t s, const int32_t* rowptr, const int32_t* col, const double* in, double* out,
                      int64_t n) {
  if (n > 0) k_mark_grow<<<grid_of(n), kMarkBlock, 0, s>>>(rowptr, col, in, out, n);
}

}  // namespace sdc
