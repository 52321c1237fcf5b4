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

// Y = A X for many right-hand sides: a work-group computes 16 rows x 32
// right-hand sides, staging 16 x 64 tiles of A and 64 x 32 tiles of X in LDS.
constexpr int MM_TM = 16, MM_TK = 64, MM_TR = 32;

__global__ __launch_bounds__(256) void k_dense_mm(const zd* __restrict__ A, int n, const zd* __restrict__ X,
                                                  zd* __restrict__ Y, int nrhs) {
  __shared__ zd As[MM_TM][MM_TK + 1];
  __shared__ zd Xs[MM_TK][MM_TR + 1];
  const int tid = threadIdx.x;
  const int row0 = blockIdx.x * MM_TM, r0 = blockIdx.y * MM_TR;
  const int lr = tid >> 4, c = tid & 15;  // row lr, right-hand sides c and c + 16
  zd acc0 = {0, 0}, acc1 = {0, 0};
  for (int k0 = 0; k0 < n; k0 += MM_TK) {
    for (int e = tid; e < MM_TM * MM_TK; e += 256) {
      const int i = e / MM_TK, k = e - i * MM_TK;
      const int gr = row0 + i, gk = k0 + k;
      As[i][k] = (gr < n && gk < n) ? A[(size_t)gr * n + gk] : zd{0, 0};
    }
    for (int e = tid; e < MM_TK * MM_TR; e += 256) {
      const int rr = e / MM_TK, k = e - rr * MM_TK;
      const int gk = k0 + k, gr = r0 + rr;
      Xs[k][rr] = (gk < n && gr < nrhs) ? X[(size_t)gr * n + gk] : zd{0, 0};
    }
    __syncthreads();
    for (int k = 0; k < MM_TK; ++k) {
      const zd a = As[lr][k];
      acc0 = acc0 + a * Xs[k][c];
      acc1 = acc1 + a * Xs[k][c + 16];
    }
    __syncthreads();
  }
  const int gr = row0 + lr;
  if (gr < n) {
    if (r0 + c < nrhs) Y[(size_t)(r0 + c) * n + gr] = acc0;
    if (r0 + c + 16 < nrhs) Y[(size_t)(r0 + c + 16) * n + gr] = acc1;
  }
}

void launch_dense_mv(const zd* A, int n, const zd* x, zd* y, int nrhs, bool many, hipStream_t s) {
  if (!many && nrhs <= 2) {
    hipLaunchKernelGGL(k_dense_mv, dim3((n + 3) / 4), dim3(256), 0, s, A, n, x, y, nrhs);
  } else {
    hipLaunchKernelGGL(k_dense_mm, dim3((n + MM_TM - 1) / MM_TM, (nrhs + MM_TR - 1) / MM_TR), dim3(256), 0, s, A,
                       n, x, y, nrhs);
  }
}

}  // namespace bamg
