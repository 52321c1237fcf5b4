// Coarsest level: the paper solves the coarsest system directly (Sec. 4).  The
// library inverts the dense coarsest operator once at setup (Gauss-Jordan
// elimination with partial pivoting, pivot = largest modulus, lowest row on
// ties) and applies the inverse as a dense matrix-vector product in every
// cycle, which is fully parallel where forward/back substitution would be a
// chain of n dependent steps.  In exact arithmetic this is the same map
// x = A_L^{-1} b as an LU solve.
#include "bamg_internal.h"

namespace bamg {

// pivot search, row swap, pivot-row scaling and saving of column k
__global__ __launch_bounds__(1024) void k_gj_pivot(zd* __restrict__ A, int n, int k, zd* __restrict__ col,
                                                   int* __restrict__ perm, int* __restrict__ flag) {
  __shared__ double bv[1024];
  __shared__ int bi[1024];
  const int tid = threadIdx.x;
  double best = -1.0;
  int besti = n;
  for (int i = k + tid; i < n; i += blockDim.x) {
    const zd a = A[(size_t)i * n + k];
    const double v = sqrt(norm2(a));
    if (v > best || (v == best && i < besti)) { best = v; besti = i; }
  }
  bv[tid] = best;
  bi[tid] = besti;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (tid < off) {
      const double v2 = bv[tid + off];
      const int i2 = bi[tid + off];
      if (v2 > bv[tid] || (v2 == bv[tid] && i2 < bi[tid])) { bv[tid] = v2; bi[tid] = i2; }
    }
    __syncthreads();
  }
  const int p = (bv[0] > 0.0) ? bi[0] : k;
  if (tid == 0) {
    perm[k] = p;
    if (!(bv[0] > 0.0)) flag[0] = 1;
  }
  if (p != k)
    for (int j = tid; j < n; j += blockDim.x) {
      const zd t = A[(size_t)k * n + j];
      A[(size_t)k * n + j] = A[(size_t)p * n + j];
      A[(size_t)p * n + j] = t;
    }
  __syncthreads();
  const zd piv = A[(size_t)k * n + k];
  const double pn = norm2(piv);
  const zd inv = pn > 0 ? zd{piv.x / pn, -piv.y / pn} : zd{0, 0};
  __syncthreads();
  for (int j = tid; j < n; j += blockDim.x) {
    const zd a = (j == k) ? zd{1.0, 0.0} : A[(size_t)k * n + j];
    A[(size_t)k * n + j] = a * inv;
  }
  for (int i = tid; i < n; i += blockDim.x) col[i] = (i == k) ? zd{0, 0} : A[(size_t)i * n + k];
}

// eliminate column k from every row but k
__global__ void k_gj_elim(zd* __restrict__ A, int n, int k, const zd* __restrict__ col) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= n || i == k) return;
  const zd f = col[i];
  const zd akj = A[(size_t)k * n + j];
  const zd aij = (j == k) ? zd{0, 0} : A[(size_t)i * n + j];
  A[(size_t)i * n + j] = aij - f * akj;
}

void launch_gj_step(zd* A, int n, int k, zd* col, int* perm, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(1024), 0, s, A, n, k, col, perm, flag);
  hipLaunchKernelGGL(k_gj_elim, dim3((n + 255) / 256, n), dim3(256), 0, s, A, n, k, col);
}

// undo the row interchanges on the columns of the inverse (last swap first)
__global__ void k_gj_unpermute(zd* __restrict__ A, int n, const int* __restrict__ perm) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  zd* Ar = A + (size_t)i * n;
  for (int k = n - 1; k >= 0; --k) {
    const int p = perm[k];
    if (p != k) {
      const zd t = Ar[k];
      Ar[k] = Ar[p];
      Ar[p] = t;
    }
  }
}

void launch_gj_unpermute(zd* A, zd* tmp, int n, const int* perm, hipStream_t s) {
  (void)tmp;
  hipLaunchKernelGGL(k_gj_unpermute, dim3((n + 63) / 64), dim3(64), 0, s, A, n, perm);
}

// y = A x, one wave per row
__global__ __launch_bounds__(256) void k_dense_mv(const zd* __restrict__ A, int n, const zd* __restrict__ x,
                                                  zd* __restrict__ y, int nrhs) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + wave;
  if (row >= n) return;
  const zd* Ar = A + (size_t)row * n;
  for (int r = 0; r < nrhs; ++r) {
    const zd* xv = x + (size_t)r * n;
    zd acc = {0, 0};
    for (int j = lane; j < n; j += 64) acc = acc + Ar[j] * xv[j];
    for (int off = 32; off > 0; off >>= 1) {
      acc.x += __shfl_xor(acc.x, off, 64);
      acc.y += __shfl_xor(acc.y, off, 64);
    }
    if (lane == 0) y[(size_t)r * n + row] = acc;
  }
}

// Y = A X for many right-hand sides: split-K tiled product.  Work-group
// (row tile, RHS tile, K quarter) computes a 32 x 32 tile over a quarter of
// K with 32-wide K chunks staged in LDS (next chunk prefetched into
// registers); the four partial tiles are summed in a fixed order by a second
// kernel (deterministic, no atomics).
constexpr int MM_T = 32, MM_K = 32, MM_SPLIT = 4;

__global__ __launch_bounds__(256) void k_dense_mm(const zd* __restrict__ A, int n, const zd* __restrict__ X,
                                                  zd* __restrict__ part, int nrhs) {
  __shared__ zd As[MM_T][MM_K + 1];
  __shared__ zd Xs[MM_K][MM_T + 1];
  const int tid = threadIdx.x;
  const int row0 = blockIdx.x * MM_T, r0 = blockIdx.y * MM_T;
  const int kq = (n + MM_SPLIT - 1) / MM_SPLIT;
  const int kbeg = blockIdx.z * kq, kend = min(n, kbeg + kq);
  const int rr = tid & 31, rq = tid >> 5;  // right-hand side rr, rows 4 rq .. 4 rq + 3
  zd acc[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
  zd pa[4], px[4];
  auto fetch = [&](int k0) {
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      const int i = e >> 5, k = e & 31;  // A tile element (row i, k) ; X tile element (rhs i, k)
      const int gk = k0 + k;
      pa[q] = (row0 + i < n && gk < kend) ? A[(size_t)(row0 + i) * n + gk] : zd{0, 0};
      px[q] = (r0 + i < nrhs && gk < kend) ? X[(size_t)(r0 + i) * n + gk] : zd{0, 0};
    }
  };
  fetch(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += MM_K) {
    __syncthreads();
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      const int i = e >> 5, k = e & 31;
      As[i][k] = pa[q];
      Xs[k][i] = px[q];
    }
    __syncthreads();
    if (k0 + MM_K < kend) fetch(k0 + MM_K);
    for (int k = 0; k < MM_K; ++k) {
      const zd xv = Xs[k][rr];
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[j] = acc[j] + As[4 * rq + j][k] * xv;
    }
  }
  if (r0 + rr < nrhs)
    for (int j = 0; j < 4; ++j) {
      const int gr = row0 + 4 * rq + j;
      if (gr < n) part[((size_t)blockIdx.z * nrhs + r0 + rr) * n + gr] = acc[j];
    }
}

__global__ void k_dense_mm_reduce(const zd* __restrict__ part, int n, int nrhs, zd* __restrict__ Y) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t tot = (size_t)n * nrhs;
  if (t >= tot) return;
  zd s = part[t];
  for (int q = 1; q < MM_SPLIT; ++q) s = s + part[(size_t)q * tot + t];
  Y[t] = s;
}

size_t dense_mm_workspace(int n, int nrhs) { return (size_t)MM_SPLIT * n * nrhs; }

void launch_dense_mv(const zd* A, int n, const zd* x, zd* y, int nrhs, bool many, zd* work, hipStream_t s) {
  if (!many && nrhs <= 2) {
    hipLaunchKernelGGL(k_dense_mv, dim3((n + 3) / 4), dim3(256), 0, s, A, n, x, y, nrhs);
  } else {
    hipLaunchKernelGGL(k_dense_mm, dim3((n + MM_T - 1) / MM_T, (nrhs + MM_T - 1) / MM_T, MM_SPLIT), dim3(256), 0, s,
                       A, n, x, work, nrhs);
    const size_t tot = (size_t)n * nrhs;
    hipLaunchKernelGGL(k_dense_mm_reduce, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, work, n, nrhs, y);
  }
}

}  // namespace bamg
