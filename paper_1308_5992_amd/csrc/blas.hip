// Vector kernels of the outer flexible GMRES (Sec. 4): batched inner products
// for classical Gram-Schmidt, the matching multi-axpy, norms, scaling.
// Reductions are deterministic: a fixed block decomposition of the index
// range gives per-block partial sums, reduced by one work-group in a fixed
// tree order (no floating-point atomics), so repeated runs are bitwise equal.
#include "bamg_internal.h"

namespace bamg {

constexpr int BT = 256;  // threads per reduction block

int blas_nblocks(size_t n) {
  size_t nb = (n + 2047) / 2048;
  if (nb < 1) nb = 1;
  if (nb > 512) nb = 512;
  return (int)nb;
}

// Short per-block chains matter more than the partial count where a launch
// holds few vectors (the single-RHS Gram-Schmidt); the slot engine's launches
// hold many and keep the coarser blocks
int blas_nblocks_fine(size_t n) {
  size_t nb = (n + 511) / 512;
  if (nb < 1) nb = 1;
  if (nb > 512) nb = 512;
  return (int)nb;
}

__device__ __forceinline__ zd block_sum(zd v, zd* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int off = BT / 2; off > 0; off >>= 1) {
    if (tid < off) sh[tid] = sh[tid] + sh[tid + off];
    __syncthreads();
  }
  return sh[0];
}

// partial[b * nv + v] = sum_{i in chunk b} conj(X_v[i]) w[i]   (w == nullptr: |X_v[i]|^2)
// X_v = X + map[v] * ldx (map == nullptr: X + v * ldx)
__global__ __launch_bounds__(BT) void k_dot_partial(const zd* __restrict__ X, size_t ldx, int nv,
                                                    const zd* __restrict__ w, size_t n, zd* __restrict__ partial,
                                                    const int* __restrict__ map) {
  __shared__ zd sh[BT];
  const int b = blockIdx.x, v = blockIdx.y, nb = gridDim.x;
  const size_t chunk = (n + nb - 1) / nb;
  const size_t lo = (size_t)b * chunk, hi = (lo + chunk < n) ? lo + chunk : n;
  const zd* xv = X + (size_t)(map ? map[v] : v) * ldx;
  zd acc = {0, 0};
  if (w) {
    for (size_t i = lo + threadIdx.x; i < hi; i += BT) acc = acc + cjmul(xv[i], w[i]);
  } else {
    for (size_t i = lo + threadIdx.x; i < hi; i += BT) acc.x += norm2(xv[i]);
  }
  const zd s = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[(size_t)b * nv + v] = s;
}

// (host_out, if not null: pinned host memory that receives a copy of out)
__global__ __launch_bounds__(BT) void k_reduce_partial(const zd* __restrict__ partial, int nb, int nv,
                                                       zd* __restrict__ out, zd* __restrict__ host_out) {
  __shared__ zd sh[BT];
  const int v = blockIdx.x;
  zd acc = {0, 0};
  for (int b = threadIdx.x; b < nb; b += BT) acc = acc + partial[(size_t)b * nv + v];
  const zd s = block_sum(acc, sh);
  if (threadIdx.x == 0) {
    out[v] = s;
    if (host_out) host_out[v] = s;
  }
}

void launch_multidot(const zd* X, size_t ldx, int nv, const zd* w, size_t n, zd* partial, zd* out,
                     hipStream_t s) {
  const int nb = blas_nblocks(n);
  hipLaunchKernelGGL(k_dot_partial, dim3(nb, nv), dim3(BT), 0, s, X, ldx, nv, w, n, partial, (const int*)nullptr);
  hipLaunchKernelGGL(k_reduce_partial, dim3(nv), dim3(BT), 0, s, partial, nb, nv, out, (zd*)nullptr);
}

void launch_norms(const zd* X, size_t ldx, int nv, size_t n, zd* partial, zd* out, hipStream_t s, const int* map,
                  bool fine) {
  const int nb = fine ? blas_nblocks_fine(n) : blas_nblocks(n);
  hipLaunchKernelGGL(k_dot_partial, dim3(nb, nv), dim3(BT), 0, s, X, ldx, nv, (const zd*)nullptr, n, partial, map);
  hipLaunchKernelGGL(k_reduce_partial, dim3(nv), dim3(BT), 0, s, partial, nb, nv, out, (zd*)nullptr);
}

// w[i] += sign * sum_v X_v[i] h[v]
__global__ void k_multiaxpy(const zd* __restrict__ X, size_t ldx, int nv, const zd* __restrict__ h, double sign,
                            zd* __restrict__ w, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  zd acc = {0, 0};
  for (int v = 0; v < nv; ++v) acc = acc + X[(size_t)v * ldx + i] * h[v];
  w[i] = w[i] + sign * acc;
}

void launch_multiaxpy(const zd* X, size_t ldx, int nv, const zd* h, double sign, zd* w, size_t n,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_multiaxpy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, X, ldx, nv, h, sign, w, n);
}

__global__ void k_normalize(zd* __restrict__ X, size_t ldx, size_t n, const zd* __restrict__ nrm) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int v = blockIdx.y;
  if (i >= n) return;
  const double q = nrm[v].x;
  if (q > 0) {
    const double s = 1.0 / sqrt(q);
    X[(size_t)v * ldx + i] = s * X[(size_t)v * ldx + i];
  }
}

void launch_normalize(zd* X, size_t ldx, int nv, size_t n, const zd* nrm, hipStream_t s) {
  hipLaunchKernelGGL(k_normalize, dim3((unsigned)((n + 255) / 256), nv), dim3(256), 0, s, X, ldx, n, nrm);
}

__global__ void k_scale_copy(const zd* __restrict__ x, zd* __restrict__ y, size_t n, double a) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i];
}

void launch_scale_copy(const zd* x, zd* y, size_t n, double alpha, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_copy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, y, n, alpha);
}

__global__ void k_sub(const zd* __restrict__ z, zd* __restrict__ x, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = x[i] - z[i];
}

void launch_sub(const zd* z, zd* x, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_sub, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, z, x, n);
}

__global__ void k_fill_zero(zd* __restrict__ x, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = zd{0, 0};
}

void launch_fill_zero(zd* x, size_t n, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n);
}

__global__ void k_zero(uint2* __restrict__ p, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = uint2{0u, 0u};
}

void launch_zero(void* p, size_t bytes, hipStream_t s) {
  const size_t n = bytes / 8;
  if (n == 0) return;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (uint2*)p, n);
}

__global__ void k_copy(const zd* __restrict__ x, zd* __restrict__ y, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i];
}

void launch_copy(const zd* x, zd* y, size_t n, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, y, n);
}

__global__ void k_check_finite(const zd* __restrict__ x, size_t n, int* __restrict__ flag) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const zd v = x[i];
    if (!isfinite(v.x) || !isfinite(v.y)) flag[0] = 1;
  }
}

void launch_check_finite(const zd* x, size_t n, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_check_finite, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n, flag);
}

// ---------------------------------------------------------------------------
// precision conversion (round to nearest even)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void cvt(const zd& a, zf& b) { b = zf{(float)a.x, (float)a.y}; }
__device__ __forceinline__ void cvt(const zf& a, zd& b) { b = zd{(double)a.x, (double)a.y}; }
__device__ __forceinline__ void cvt(const zd& a, hcx& b) {
  b.x = __float2half_rn((float)a.x);
  b.y = __float2half_rn((float)a.y);
}
__device__ __forceinline__ void cvt(const zd& a, bcx& b) {
  b.x = __float2bfloat16((float)a.x);
  b.y = __float2bfloat16((float)a.y);
}

template <typename Tin, typename Tout>
__global__ void k_convert(const Tin* __restrict__ in, Tout* __restrict__ out, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) cvt(in[i], out[i]);
}

template <typename Tin, typename Tout>
void launch_convert(const Tin* in, Tout* out, size_t n, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL((k_convert<Tin, Tout>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, out, n);
}
// out = in converted, and zero_out = 0 (the same n entries): the mixed
// preconditioner's input and its zero initial guess in one launch
template <typename Tin, typename Tout>
__global__ void k_convert_zero(const Tin* __restrict__ in, Tout* __restrict__ out, Tout* __restrict__ zero_out,
                               size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    cvt(in[i], out[i]);
    zero_out[i] = Tout{0, 0};
  }
}
void launch_convert_zero(const zd* in, zf* out, zf* zero_out, size_t n, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL((k_convert_zero<zd, zf>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, out, zero_out, n);
}
template void launch_convert<zd, zf>(const zd*, zf*, size_t, hipStream_t);
template void launch_convert<zf, zd>(const zf*, zd*, size_t, hipStream_t);
template void launch_convert<zd, hcx>(const zd*, hcx*, size_t, hipStream_t);
template void launch_convert<zd, bcx>(const zd*, bcx*, size_t, hipStream_t);

// ---------------------------------------------------------------------------
// Batched forms for R right-hand sides.  Basis vector v of right-hand side r
// lives at X + (v*R + r)*n (layout [v][r][n]); w_r at W + r*n; coefficient
// arrays have a stride of 64 per right-hand side.  Each right-hand side uses
// exactly the block decomposition of the single form, so its results do not
// depend on R.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BT) void k_bdot_partial(const zd* __restrict__ X, int R, const zd* __restrict__ W,
                                                     size_t n, zd* __restrict__ partial) {
  __shared__ zd sh[BT];
  const int b = blockIdx.x, v = blockIdx.y, r = blockIdx.z, nb = gridDim.x;
  const size_t chunk = (n + nb - 1) / nb;
  const size_t lo = (size_t)b * chunk, hi = (lo + chunk < n) ? lo + chunk : n;
  const zd* xv = X + ((size_t)v * R + r) * n;
  const zd* wv = W + (size_t)r * n;
  zd acc = {0, 0};
  for (size_t i = lo + threadIdx.x; i < hi; i += BT) acc = acc + cjmul_fixed(xv[i], wv[i]);
  const zd s = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[((size_t)r * nb + b) * 64 + v] = s;
}

__global__ __launch_bounds__(BT) void k_breduce(const zd* __restrict__ partial, int nb, zd* __restrict__ out,
                                                zd* __restrict__ host_out) {
  __shared__ zd sh[BT];
  const int v = blockIdx.x, r = blockIdx.y;
  zd acc = {0, 0};
  for (int b = threadIdx.x; b < nb; b += BT) acc = acc + partial[((size_t)r * nb + b) * 64 + v];
  const zd s = block_sum(acc, sh);
  if (threadIdx.x == 0) {
    out[(size_t)r * 64 + v] = s;
    if (host_out) host_out[(size_t)r * 64 + v] = s;
  }
}

void launch_bmultidot(const zd* X, int nv, const zd* W, size_t n, int R, zd* partial, zd* out, hipStream_t s,
                      zd* host_out) {
  const int nb = blas_nblocks_fine(n);
  hipLaunchKernelGGL(k_bdot_partial, dim3(nb, nv, R), dim3(BT), 0, s, X, R, W, n, partial);
  hipLaunchKernelGGL(k_breduce, dim3(nv, R), dim3(BT), 0, s, partial, nb, out, host_out);
}

__global__ void k_bmultiaxpy(const zd* __restrict__ X, int nv, int R, const zd* __restrict__ h, double sign,
                             zd* __restrict__ W, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (i >= n) return;
  zd acc = {0, 0};
  for (int v = 0; v < nv; ++v) acc = acc + cmul_fixed(X[((size_t)v * R + r) * n + i], h[(size_t)r * 64 + v]);
  W[(size_t)r * n + i] = W[(size_t)r * n + i] + sign * acc;
}

void launch_bmultiaxpy(const zd* X, int nv, const zd* h, double sign, zd* W, size_t n, int R, hipStream_t s) {
  hipLaunchKernelGGL(k_bmultiaxpy, dim3((unsigned)((n + 255) / 256), R), dim3(256), 0, s, X, nv, R, h, sign, W, n);
}

// The partial inner products of one chunk [lo, hi) of a right-hand side's
// w with X_0..X_{nd-1} (X_v at X + (v R + r) n), for work-groups of PD_BT
// threads: thread t holds w at lo + t + k PD_BT in wl[k], accumulates
// conj(X_v) w over its entries in order from zero, and the work-group sums
// the threads by the halving tree (t + off into t, off = PD_BT / 2 ... 1),
// PD_VC vectors per tree; partial[(r nb + b) 64 + v]: the order of
// k_bdot_partial.
constexpr int PD_BT = 256, PD_VC = 8;
template <int E>
__device__ __forceinline__ void block_partial_dots(const zd* __restrict__ X, int R, int r, size_t n, size_t lo,
                                                   size_t hi, const zd (&wl)[E], int nd, zd (*sh)[PD_BT],
                                                   zd* __restrict__ partial, int nb, int b) {
  const int tid = threadIdx.x;
  for (int v0 = 0; v0 < nd; v0 += PD_VC) {
#pragma unroll
    for (int q = 0; q < PD_VC; ++q) {
      const int v = v0 + q;
      zd acc = {0, 0};
      if (v < nd) {
        const zd* xv = X + ((size_t)v * R + r) * n;
#pragma unroll
        for (int k = 0; k < E; ++k) {
          const size_t i = lo + tid + (size_t)k * PD_BT;
          if (i < hi) acc = acc + cjmul_fixed(xv[i], wl[k]);
        }
      }
      sh[q][tid] = acc;
    }
    __syncthreads();
    for (int off = PD_BT / 2; off > 0; off >>= 1) {
      if (tid < off) {
#pragma unroll
        for (int q = 0; q < PD_VC; ++q) sh[q][tid] = sh[q][tid] + sh[q][tid + off];
      }
      __syncthreads();
    }
    if (tid < PD_VC && v0 + tid < nd) partial[((size_t)r * nb + b) * 64 + v0 + tid] = sh[tid][0];
    __syncthreads();
  }
}

// A Gram-Schmidt step and the reduction after it in one launch: block b of
// right-hand side r updates its chunk of w_r by the multi-axpy
// (k_bmultiaxpy's arithmetic), then forms from the updated chunk the partial
// inner products with X_0..X_{nd-1} (nd > 0; k_bdot_partial's block
// decomposition, per-thread order and tree; block_partial_dots) or the
// partial squared norm (nd = 0; partial[b R + r], the layout of
// k_dot_partial).  A chunk holds at most BAX_E entries per thread.
constexpr int BAX_E = 4;
__global__ __launch_bounds__(BT) void k_baxpy_dot(const zd* __restrict__ X, int nv, int R, const zd* __restrict__ h,
                                                  double sign, zd* __restrict__ W, size_t n, int nd,
                                                  zd* __restrict__ partial) {
  __shared__ zd sh[PD_VC][PD_BT];
  const int b = blockIdx.x, r = blockIdx.y, nb = gridDim.x, tid = threadIdx.x;
  const size_t chunk = (n + nb - 1) / nb;
  const size_t lo = (size_t)b * chunk, hi = (lo + chunk < n) ? lo + chunk : n;
  zd* wv = W + (size_t)r * n;
  zd wl[BAX_E];
#pragma unroll
  for (int k = 0; k < BAX_E; ++k) {
    const size_t i = lo + tid + (size_t)k * BT;
    wl[k] = zd{0, 0};
    if (i < hi) {
      zd acc = {0, 0};
      for (int v = 0; v < nv; ++v) acc = acc + cmul_fixed(X[((size_t)v * R + r) * n + i], h[(size_t)r * 64 + v]);
      wl[k] = wv[i] + sign * acc;
      wv[i] = wl[k];
    }
  }
  if (nd == 0) {
    zd acc = {0, 0};
#pragma unroll
    for (int k = 0; k < BAX_E; ++k)
      if (lo + tid + (size_t)k * BT < hi) acc.x = acc.x + fma(wl[k].x, wl[k].x, wl[k].y * wl[k].y);
    const zd s = block_sum(acc, sh[0]);
    if (tid == 0) partial[(size_t)b * R + r] = s;
    return;
  }
  block_partial_dots<BAX_E>(X, R, r, n, lo, hi, wl, nd, sh, partial, nb, b);
}

bool baxpy_dot_applies(size_t n) {
  const int nb = blas_nblocks_fine(n);
  return (n + nb - 1) / nb <= (size_t)BAX_E * BT;
}

bool launch_baxpy_dot(const zd* X, int nv, const zd* h, double sign, zd* W, size_t n, int R, int nd, zd* partial,
                      zd* out, hipStream_t s, zd* host_out) {
  const int nb = blas_nblocks_fine(n);
  if (!baxpy_dot_applies(n) || nd < 0 || nd > 64) return false;
  hipLaunchKernelGGL(k_baxpy_dot, dim3(nb, R), dim3(BT), 0, s, X, nv, R, h, sign, W, n, nd, partial);
  if (nd > 0) hipLaunchKernelGGL(k_breduce, dim3(nd, R), dim3(BT), 0, s, partial, nb, out, host_out);
  else if (out) hipLaunchKernelGGL(k_reduce_partial, dim3(R), dim3(BT), 0, s, partial, nb, R, out, host_out);
  return true;
}

__global__ void k_bscale(const zd* __restrict__ x, zd* __restrict__ y, size_t n, const double* __restrict__ c) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (i < n) y[(size_t)r * n + i] = c[r] * x[(size_t)r * n + i];
}

void launch_bscale(const zd* x, zd* y, size_t n, int R, const double* c, hipStream_t s) {
  hipLaunchKernelGGL(k_bscale, dim3((unsigned)((n + 255) / 256), R), dim3(256), 0, s, x, y, n, c);
}

// y = x / sqrt(nrm2.x): the next Arnoldi vector from the squared norm left
// on the device (the host's 1 / sqrt, correctly rounded both ways); a zero
// norm (an exhausted Krylov space, where the host stops and any iteration
// queued ahead goes unused) gives y = 0 rather than NaN
__global__ void k_bscale_rnorm(const zd* __restrict__ x, zd* __restrict__ y, size_t n, const zd* __restrict__ nrm2) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double q = nrm2[0].x;
  if (i < n) y[i] = q > 0 ? (1.0 / sqrt(q)) * x[i] : zd{0, 0};
}

// One right-hand side: |w|^2 summed from the nb block partials in every
// work-group with k_reduce_partial's per-thread order and tree (block 0
// writes it to out and host_out), then y = w / |w| over the work-group's
// chunk with k_bscale_rnorm's arithmetic: the norm and the next Arnoldi
// vector in one launch, the same bits as the two
constexpr int NS_E = 4;
__global__ __launch_bounds__(BT) void k_norm_scale(const zd* __restrict__ partial, int nb, const zd* __restrict__ w,
                                                   zd* __restrict__ y, size_t n, zd* __restrict__ out,
                                                   zd* __restrict__ host_out) {
  __shared__ zd sh[BT];
  zd acc = {0, 0};
  for (int b = threadIdx.x; b < nb; b += BT) acc = acc + partial[b];
  const zd nrm = block_sum(acc, sh);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    out[0] = nrm;
    if (host_out) host_out[0] = nrm;
  }
  const double q = nrm.x;
#pragma unroll
  for (int k = 0; k < NS_E; ++k) {
    const size_t i = ((size_t)blockIdx.x * NS_E + k) * BT + threadIdx.x;
    if (i < n) y[i] = q > 0 ? (1.0 / sqrt(q)) * w[i] : zd{0, 0};
  }
}

void launch_norm_scale(const zd* partial, const zd* w, zd* y, size_t n, zd* out, zd* host_out, hipStream_t s) {
  const size_t per = (size_t)NS_E * BT;
  hipLaunchKernelGGL(k_norm_scale, dim3((unsigned)((n + per - 1) / per)), dim3(BT), 0, s, partial,
                     blas_nblocks_fine(n), w, y, n, out, host_out);
}

void launch_bscale_rnorm(const zd* x, zd* y, size_t n, const zd* nrm2, hipStream_t s) {
  hipLaunchKernelGGL(k_bscale_rnorm, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, y, n, nrm2);
}

__global__ void k_blincomb(const zd* __restrict__ Z, int nq, int R, const zd* __restrict__ y, zd* __restrict__ x,
                           size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (i >= n) return;
  zd acc = {0, 0};
  for (int q = 0; q < nq; ++q) acc = acc + Z[((size_t)q * R + r) * n + i] * y[(size_t)r * 64 + q];
  x[(size_t)r * n + i] = x[(size_t)r * n + i] + acc;
}

void launch_blincomb(const zd* Z, int nq, const zd* y, zd* x, size_t n, int R, hipStream_t s) {
  if (nq <= 0) return;
  hipLaunchKernelGGL(k_blincomb, dim3((unsigned)((n + 255) / 256), R), dim3(256), 0, s, Z, nq, R, y, x, n);
}

// ---------------------------------------------------------------------------
// Slot-mapped forms for continuous batching.  Entry a of a launch works on the
// right-hand side held in slot slot[a]; vector v of that slot's basis lives at
// X + slot[a] * lds + v * ldv, and only its first cnt[a] vectors are used.
// Gathered per-launch vectors (w, the inputs and outputs of the cycle) are
// contiguous at W + a * n.  Each entry repeats exactly the arithmetic of the
// unmapped batched forms above (same block decomposition, same accumulation
// order), so a right-hand side's results depend neither on its slot nor on
// the other entries of the launch.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BT) void k_sdot_partial(const zd* __restrict__ X, size_t lds, size_t ldv,
                                                     const int* __restrict__ slot, const int* __restrict__ cnt,
                                                     const zd* __restrict__ W, size_t n, zd* __restrict__ partial) {
  __shared__ zd sh[BT];
  const int b = blockIdx.x, v = blockIdx.y, a = blockIdx.z, nb = gridDim.x;
  if (v >= cnt[a]) return;  // uniform over the block
  const size_t chunk = (n + nb - 1) / nb;
  const size_t lo = (size_t)b * chunk, hi = (lo + chunk < n) ? lo + chunk : n;
  const zd* xv = X + (size_t)slot[a] * lds + (size_t)v * ldv;
  const zd* wv = W + (size_t)a * n;
  zd acc = {0, 0};
  for (size_t i = lo + threadIdx.x; i < hi; i += BT) acc = acc + cjmul(xv[i], wv[i]);
  const zd s = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[((size_t)a * nb + b) * 64 + v] = s;
}

__global__ __launch_bounds__(BT) void k_sreduce(const zd* __restrict__ partial, int nb, const int* __restrict__ cnt,
                                                zd* __restrict__ out) {
  __shared__ zd sh[BT];
  const int v = blockIdx.x, a = blockIdx.y;
  if (v >= cnt[a]) return;
  zd acc = {0, 0};
  for (int b = threadIdx.x; b < nb; b += BT) acc = acc + partial[((size_t)a * nb + b) * 64 + v];
  const zd s = block_sum(acc, sh);
  if (threadIdx.x == 0) out[(size_t)a * 64 + v] = s;
}

void launch_smultidot(const zd* X, size_t lds, size_t ldv, const int* slot, const int* cnt, int maxcnt, const zd* W,
                      size_t n, int A, zd* partial, zd* out, hipStream_t s) {
  if (A <= 0 || maxcnt <= 0) return;
  const int nb = blas_nblocks(n);
  hipLaunchKernelGGL(k_sdot_partial, dim3(nb, maxcnt, A), dim3(BT), 0, s, X, lds, ldv, slot, cnt, W, n, partial);
  hipLaunchKernelGGL(k_sreduce, dim3(maxcnt, A), dim3(BT), 0, s, partial, nb, cnt, out);
}

__global__ void k_smultiaxpy(const zd* __restrict__ X, size_t lds, size_t ldv, const int* __restrict__ slot,
                             const int* __restrict__ cnt, const zd* __restrict__ h, double sign, zd* __restrict__ W,
                             size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int a = blockIdx.y;
  if (i >= n) return;
  const zd* xs = X + (size_t)slot[a] * lds;
  const int nv = cnt[a];
  zd acc = {0, 0};
  for (int v = 0; v < nv; ++v) acc = acc + xs[(size_t)v * ldv + i] * h[(size_t)a * 64 + v];
  W[(size_t)a * n + i] = W[(size_t)a * n + i] + sign * acc;
}

void launch_smultiaxpy(const zd* X, size_t lds, size_t ldv, const int* slot, const int* cnt, const zd* h, double sign,
                       zd* W, size_t n, int A, hipStream_t s) {
  if (A <= 0) return;
  hipLaunchKernelGGL(k_smultiaxpy, dim3((unsigned)((n + 255) / 256), A), dim3(256), 0, s, X, lds, ldv, slot, cnt, h,
                     sign, W, n);
}

// x_{slot[a]} += sum_{q < cnt[a]} Z_{slot[a], q} y[a][q]   (x slot-major, stride n)
__global__ void k_slincomb(const zd* __restrict__ Z, size_t lds, size_t ldv, const int* __restrict__ slot,
                           const int* __restrict__ cnt, const zd* __restrict__ y, zd* __restrict__ x, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int a = blockIdx.y;
  if (i >= n) return;
  const zd* zs = Z + (size_t)slot[a] * lds;
  const int nq = cnt[a];
  zd acc = {0, 0};
  for (int q = 0; q < nq; ++q) acc = acc + zs[(size_t)q * ldv + i] * y[(size_t)a * 64 + q];
  zd* xs = x + (size_t)slot[a] * n;
  xs[i] = xs[i] + acc;
}

void launch_slincomb(const zd* Z, size_t lds, size_t ldv, const int* slot, const int* cnt, const zd* y, zd* x,
                     size_t n, int A, hipStream_t s) {
  if (A <= 0) return;
  hipLaunchKernelGGL(k_slincomb, dim3((unsigned)((n + 255) / 256), A), dim3(256), 0, s, Z, lds, ldv, slot, cnt, y, x,
                     n);
}

// Y_a = X_{slot[a], j[a]}   (j == nullptr: vector 0)
__global__ void k_sgather(const zd* __restrict__ X, size_t lds, size_t ldv, const int* __restrict__ slot,
                          const int* __restrict__ j, zd* __restrict__ Y, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int a = blockIdx.y;
  if (i >= n) return;
  Y[(size_t)a * n + i] = X[(size_t)slot[a] * lds + (size_t)(j ? j[a] : 0) * ldv + i];
}

void launch_sgather(const zd* X, size_t lds, size_t ldv, const int* slot, const int* j, zd* Y, size_t n, int A,
                    hipStream_t s) {
  if (A <= 0) return;
  hipLaunchKernelGGL(k_sgather, dim3((unsigned)((n + 255) / 256), A), dim3(256), 0, s, X, lds, ldv, slot, j, Y, n);
}

// X_{slot[a], j[a]} = c[a] * Y_{src[a]}   (c == nullptr: plain copy; src == nullptr: a;
// Y_k at Y + k * ldy)
__global__ void k_sscatter(const zd* __restrict__ Y, size_t ldy, const int* __restrict__ src, zd* __restrict__ X,
                           size_t lds, size_t ldv, const int* __restrict__ slot, const int* __restrict__ j,
                           const double* __restrict__ c, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int a = blockIdx.y;
  if (i >= n) return;
  const zd v = Y[(size_t)(src ? src[a] : a) * ldy + i];
  X[(size_t)slot[a] * lds + (size_t)(j ? j[a] : 0) * ldv + i] = c ? c[a] * v : v;
}

void launch_sscatter(const zd* Y, size_t ldy, const int* src, zd* X, size_t lds, size_t ldv, const int* slot,
                     const int* j, const double* c, size_t n, int A, hipStream_t s) {
  if (A <= 0) return;
  hipLaunchKernelGGL(k_sscatter, dim3((unsigned)((n + 255) / 256), A), dim3(256), 0, s, Y, ldy, src, X, lds, ldv,
                     slot, j, c, n);
}

}  // namespace bamg
