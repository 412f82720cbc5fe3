// Vector helpers (power iteration, thresholds, fills) and the leaf back
// substitution of the solve.
#include "kernels_common.h"
#include "kernels.h"

namespace hq {
// x <- z / |z|, out[0] = |z|  (one block per item; x or out may be null)
__global__ void __launch_bounds__(1024) k_normalize(const VecJob* __restrict__ items, int first) {
  __shared__ double red[16];
  const VecJob it = items[first + blockIdx.x];
  const double* z = it.z;
  const int64_t n = it.n;
  // sixteen loads in flight per thread (a plain loop waits for every load)
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int64_t i = threadIdx.x;
  for (; i + 15 * 1024 < n; i += 16 * 1024) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = z[i + u * 1024];
#pragma unroll
    for (int u = 0; u < 16; u += 4) {
      s0 += v[u] * v[u];
      s1 += v[u + 1] * v[u + 1];
      s2 += v[u + 2] * v[u + 2];
      s3 += v[u + 3] * v[u + 3];
    }
  }
  for (; i < n; i += 1024) s0 += z[i] * z[i];
  double s = (s0 + s1) + (s2 + s3);
  s = gsum(s, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < 16; ++i) t += red[i];
  const double nrm = sqrt(t);
  if (it.x != nullptr) {
    const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
    int64_t j = threadIdx.x;
    for (; j + 15 * 1024 < n; j += 16 * 1024) {
      double v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = z[j + u * 1024];
#pragma unroll
      for (int u = 0; u < 16; ++u) it.x[j + u * 1024] = v[u] * inv;
    }
    for (; j < n; j += 1024) it.x[j] = z[j] * inv;
  }
  if (threadIdx.x == 0 && it.out != nullptr) it.out[0] = nrm;
}

// thresholds of one factorisation: x = [|A|_2, eps*|A|_2, eps] with eps = d0 and
// |A|_2 = d1 if d1 > 0, else the estimate already in x[0]  (one thread per item)
__global__ void k_set_scal(const VecJob* __restrict__ items, int first, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const VecJob it = items[first + i];
  const double a = it.d1 > 0.0 ? it.d1 : it.x[0];
  it.x[0] = a;
  it.x[1] = it.d0 * a;
  it.x[2] = it.d0;
}

// x[0:n] = d0, one block per item
__global__ void k_fill_items(const VecJob* __restrict__ items, int first) {
  const VecJob it = items[first + blockIdx.x];
  for (int64_t i = threadIdx.x; i < it.n; i += blockDim.x) it.x[i] = it.d0;
}

__global__ void k_fill(double* x, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

__global__ void k_zero_i32(int* x, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0;
}

// Back substitution with one upper triangular leaf: X <- R^{-1} X (m x nrhs).
__global__ void __launch_bounds__(NT_MM) k_leaf_trsm(const double* __restrict__ D, int m, int ld,
                                                      double* X, int ldx, int nrhs) {
  __shared__ double xs[MAXLEAF];
  __shared__ double red[4];
  const int c = blockIdx.x;  // one column per block
  if (c >= nrhs) return;
  double* x = X + (int64_t)c * ldx;
  for (int r = threadIdx.x; r < m; r += NT_MM) xs[r] = x[r];
  __syncthreads();
  for (int i = m - 1; i >= 0; --i) {
    double s = 0.0;
    for (int j = i + 1 + threadIdx.x; j < m; j += NT_MM) s += D[i + (int64_t)j * ld] * xs[j];
    s = gsum(s, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) xs[i] = (xs[i] - (red[0] + red[1] + red[2] + red[3])) / D[i + (int64_t)i * ld];
    __syncthreads();
  }
  for (int r = threadIdx.x; r < m; r += NT_MM) x[r] = xs[r];
}

// X(c0_j + i, col) = B(r0_j + i, col) for i < n_j: the pivot rows of each leaf
// (runs[3 j] = r0_j, runs[3 j + 1] = c0_j, runs[3 j + 2] = n_j); block (j, col
// group), columns col, col + gridDim.y, ...
__global__ void __launch_bounds__(NT_MM) k_pivot_rows(const int* __restrict__ runs, int nrun, const double* B,
                                                      int ldb, double* X, int ldx, int ncols) {
  const int j = blockIdx.x;
  if (j >= nrun) return;
  const int r0 = runs[3 * j], c0 = runs[3 * j + 1], nj = runs[3 * j + 2];
  for (int col = blockIdx.y; col < ncols; col += gridDim.y)
    for (int i = threadIdx.x; i < nj; i += NT_MM)
      X[c0 + i + (int64_t)col * ldx] = B[r0 + i + (int64_t)col * ldb];
}

// Row runs between column-major arrays: one block per run, every column.
__global__ void __launch_bounds__(NT_MM) k_rows(const RowJob* __restrict__ items, int first) {
  const RowJob J = items[first + blockIdx.x];
  const int nc = J.ncols_dev ? *J.ncols_dev : J.ncols;
  const int64_t total = (int64_t)J.rows * nc;
  for (int64_t e = threadIdx.x; e < total; e += NT_MM) {
    const int r = (int)(e % J.rows), c = (int)(e / J.rows);
    J.dst[J.dst_r0 + r + (int64_t)c * J.ldd] = J.src[J.src_r0 + r + (int64_t)c * J.lds];
  }
}

}  // namespace hq
