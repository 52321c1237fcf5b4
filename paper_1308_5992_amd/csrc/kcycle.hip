// Krylov-accelerated coarse visits of the K-cycle option: two steps of
// flexible GCR on a coarse system A_c x = r0 from x = 0, each preconditioned
// by one cycle from level c,
//   z1 = M r0, w1 = A z1, a1 = <w1, r0> / <w1, w1>, x = a1 z1, r1 = r0 - a1 w1,
//   z2 = M r1, w2 = A z2, beta = <w1, w2> / <w1, w1>, w2 -= beta w1, z2 -= beta z1,
//   a2 = <w2, r1> / <w2, w2>, x += a2 z2
// (<u, v> = sum conj(u_i) v_i).  The cycles and operator applications are the
// level kernels; this file holds the inner products, the coefficients and the
// vector updates.  Every reduction has a block decomposition that depends on n
// only and is summed in a fixed order, and every right-hand side of a launch
// is reduced on its own, so a right-hand side's coefficients do not depend on
// the batch.  Sums and coefficients are FP64 for both vector types (FP32
// vectors of the mixed cycle are widened exactly); the coefficients stay on
// the device, so a visit is a fixed launch sequence that a graph can capture.
#include "bamg_internal.h"

namespace bamg {

namespace {

constexpr int KT = 256;  // threads per reduction block

template <typename T>
__device__ __forceinline__ zd wide(cx<T> v) {
  return zd{(double)v.x, (double)v.y};
}

template <typename T>
__device__ __forceinline__ cx<T> narrow(zd v) {
  return cx<T>{(T)v.x, (T)v.y};
}

// two sums over the block in a fixed tree order
__device__ __forceinline__ void block_sum2(zd& a, zd& b, zd* sh) {
  const int tid = threadIdx.x;
  sh[tid] = a;
  sh[KT + tid] = b;
  __syncthreads();
  for (int off = KT / 2; off > 0; off >>= 1) {
    if (tid < off) {
      sh[tid] = sh[tid] + sh[tid + off];
      sh[KT + tid] = sh[KT + tid] + sh[KT + tid + off];
    }
    __syncthreads();
  }
  a = sh[0];
  b = sh[KT];
}

// partial[(b R + r) 2 + 0] = sum over chunk b of conj(A_r) X1_r, [.. + 1] likewise with X2_r (0 if X2 is NULL)
template <typename T>
__global__ __launch_bounds__(KT) void k_kdots(const cx<T>* __restrict__ A, const cx<T>* __restrict__ X1,
                                              const cx<T>* __restrict__ X2, size_t n, zd* __restrict__ partial) {
  __shared__ zd sh[2 * KT];
  const int b = blockIdx.x, r = blockIdx.y, nb = gridDim.x, R = gridDim.y;
  const size_t chunk = (n + nb - 1) / nb;
  const size_t lo = (size_t)b * chunk, hi = (lo + chunk < n) ? lo + chunk : n;
  const size_t off = (size_t)r * n;
  zd s1 = {0, 0}, s2 = {0, 0};
  for (size_t i = lo + threadIdx.x; i < hi; i += KT) {
    const zd a = wide(A[off + i]);
    s1 = s1 + cjmul(a, wide(X1[off + i]));
    if (X2) s2 = s2 + cjmul(a, wide(X2[off + i]));
  }
  block_sum2(s1, s2, sh);
  if (threadIdx.x == 0) {
    partial[((size_t)b * R + r) * 2] = s1;
    partial[((size_t)b * R + r) * 2 + 1] = s2;
  }
}

// W -= beta W', Z -= beta Z' (beta = coef[4 r + 2]), then the partial sums of
// conj(W) W and conj(W) X2 with the updated W
template <typename T>
__global__ __launch_bounds__(KT) void k_korth_dots(cx<T>* __restrict__ W, const cx<T>* __restrict__ Wp,
                                                   cx<T>* __restrict__ Z, const cx<T>* __restrict__ Zp,
                                                   const cx<T>* __restrict__ X2, const zd* __restrict__ coef, size_t n,
                                                   zd* __restrict__ partial) {
  __shared__ zd sh[2 * KT];
  const int b = blockIdx.x, r = blockIdx.y, nb = gridDim.x, R = gridDim.y;
  const size_t chunk = (n + nb - 1) / nb;
  const size_t lo = (size_t)b * chunk, hi = (lo + chunk < n) ? lo + chunk : n;
  const size_t off = (size_t)r * n;
  const zd beta = coef[4 * r + 2];
  zd s1 = {0, 0}, s2 = {0, 0};
  for (size_t i = lo + threadIdx.x; i < hi; i += KT) {
    const zd w = wide(W[off + i]) - beta * wide(Wp[off + i]);
    const zd z = wide(Z[off + i]) - beta * wide(Zp[off + i]);
    const cx<T> wn = narrow<T>(w);
    W[off + i] = wn;
    Z[off + i] = narrow<T>(z);
    const zd a = wide(wn);
    s1.x += norm2(a);
    s2 = s2 + cjmul(a, wide(X2[off + i]));
  }
  block_sum2(s1, s2, sh);
  if (threadIdx.x == 0) {
    partial[((size_t)b * R + r) * 2] = s1;
    partial[((size_t)b * R + r) * 2 + 1] = s2;
  }
}

// one work-group per right-hand side: d1, d2 = the fixed-order sums of the
// partials, then the coefficient of `mode`:
//   0: rho1 = Re d1 -> coef[4r+1], a1 = d2 / rho1 -> coef[4r]
//   1: beta = d1 / rho1 -> coef[4r+2]
//   2: a2 = d2 / Re d1 -> coef[4r+3]
// a vanishing denominator gives a zero coefficient (the step adds nothing)
__global__ __launch_bounds__(KT) void k_kcoef(const zd* __restrict__ partial, int nb, int mode, zd* __restrict__ coef) {
  __shared__ zd sh[2 * KT];
  const int r = blockIdx.x, R = gridDim.x;
  zd d1 = {0, 0}, d2 = {0, 0};
  for (int b = threadIdx.x; b < nb; b += KT) {
    d1 = d1 + partial[((size_t)b * R + r) * 2];
    d2 = d2 + partial[((size_t)b * R + r) * 2 + 1];
  }
  block_sum2(d1, d2, sh);
  if (threadIdx.x != 0) return;
  if (mode == 0) {
    const double rho = d1.x;
    coef[4 * r + 1] = zd{rho, 0.0};
    coef[4 * r] = rho > 0.0 ? cdiv_real(d2, rho) : zd{0, 0};
  } else if (mode == 1) {
    const double rho = coef[4 * r + 1].x;
    coef[4 * r + 2] = rho > 0.0 ? cdiv_real(d1, rho) : zd{0, 0};
  } else {
    const double rho = d1.x;
    coef[4 * r + 3] = rho > 0.0 ? cdiv_real(d2, rho) : zd{0, 0};
  }
}

// x = a1 z1, r1 = r0 - a1 w1
template <typename T>
__global__ void k_kstep1(const cx<T>* __restrict__ z1, const cx<T>* __restrict__ w1, const cx<T>* __restrict__ r0,
                         const zd* __restrict__ coef, cx<T>* __restrict__ x, cx<T>* __restrict__ r1, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (i >= n) return;
  const size_t k = (size_t)r * n + i;
  const zd a1 = coef[4 * r];
  x[k] = narrow<T>(a1 * wide(z1[k]));
  r1[k] = narrow<T>(wide(r0[k]) - a1 * wide(w1[k]));
}

// x += a2 z2
template <typename T>
__global__ void k_kstep3(const cx<T>* __restrict__ z2, const zd* __restrict__ coef, cx<T>* __restrict__ x, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (i >= n) return;
  const size_t k = (size_t)r * n + i;
  x[k] = narrow<T>(wide(x[k]) + coef[4 * r + 3] * wide(z2[k]));
}

}  // namespace

int kcycle_nblocks(size_t n) { return blas_nblocks(n); }

template <typename T>
void launch_kdots(const cx<T>* A, const cx<T>* X1, const cx<T>* X2, size_t n, int R, zd* partial, hipStream_t s) {
  hipLaunchKernelGGL(k_kdots<T>, dim3(kcycle_nblocks(n), R), dim3(KT), 0, s, A, X1, X2, n, partial);
}

template <typename T>
void launch_korth_dots(cx<T>* W, const cx<T>* Wp, cx<T>* Z, const cx<T>* Zp, const cx<T>* X2, const zd* coef,
                       size_t n, int R, zd* partial, hipStream_t s) {
  hipLaunchKernelGGL(k_korth_dots<T>, dim3(kcycle_nblocks(n), R), dim3(KT), 0, s, W, Wp, Z, Zp, X2, coef, n,
                     partial);
}

void launch_kcoef(const zd* partial, size_t n, int R, int mode, zd* coef, hipStream_t s) {
  hipLaunchKernelGGL(k_kcoef, dim3(R), dim3(KT), 0, s, partial, kcycle_nblocks(n), mode, coef);
}

template <typename T>
void launch_kstep1(const cx<T>* z1, const cx<T>* w1, const cx<T>* r0, const zd* coef, cx<T>* x, cx<T>* r1, size_t n,
                   int R, hipStream_t s) {
  hipLaunchKernelGGL(k_kstep1<T>, dim3((unsigned)((n + 255) / 256), R), dim3(256), 0, s, z1, w1, r0, coef, x, r1, n);
}

template <typename T>
void launch_kstep3(const cx<T>* z2, const zd* coef, cx<T>* x, size_t n, int R, hipStream_t s) {
  hipLaunchKernelGGL(k_kstep3<T>, dim3((unsigned)((n + 255) / 256), R), dim3(256), 0, s, z2, coef, x, n);
}

template void launch_kdots<double>(const zd*, const zd*, const zd*, size_t, int, zd*, hipStream_t);
template void launch_kdots<float>(const zf*, const zf*, const zf*, size_t, int, zd*, hipStream_t);
template void launch_korth_dots<double>(zd*, const zd*, zd*, const zd*, const zd*, const zd*, size_t, int, zd*,
                                        hipStream_t);
template void launch_korth_dots<float>(zf*, const zf*, zf*, const zf*, const zf*, const zd*, size_t, int, zd*,
                                       hipStream_t);
template void launch_kstep1<double>(const zd*, const zd*, const zd*, const zd*, zd*, zd*, size_t, int, hipStream_t);
template void launch_kstep1<float>(const zf*, const zf*, const zf*, const zd*, zf*, zf*, size_t, int, hipStream_t);
template void launch_kstep3<double>(const zd*, const zd*, zd*, size_t, int, hipStream_t);
template void launch_kstep3<float>(const zf*, const zd*, zf*, size_t, int, hipStream_t);

}  // namespace bamg
