// Coarsest level: the paper solves the coarsest system directly (Sec. 4).  The
// library inverts the dense coarsest operator once at setup (blocked
// Gauss-Jordan elimination with partial pivoting, pivot = largest modulus,
// lowest row on ties) and applies the inverse as a dense matrix-vector (or
// matrix-matrix) product in every cycle, which is fully parallel where
// forward/back substitution would be a chain of n dependent steps.  In exact
// arithmetic this is the same map x = A_L^{-1} b as an LU solve.
#include "bamg_internal.h"

namespace bamg {

// Blocked Gauss-Jordan elimination.  The b pivot steps k0 .. k0+b-1 of the
// unblocked elimination act on the panel columns K = [k0, k0+b) on their own
// (a row operation with pivot row k changes column j by a multiple of the
// pivot row's entry in column j), so the panel is eliminated first, one pivot
// step per pair of launches, with the pivot search and row interchanges, into
//     A[K][K] <- inv(A11),   A[I][K] <- -A[I][K] inv(A11)   (I = rows not in K).
// The same b steps act on every other column j as
//     A[K][j] <- inv(A11) A[K][j],   A[I][j] <- A[I][j] - A[I][K] inv(A11) A[K][j],
// i.e. with T = A[K][j] (after the interchanges) and the eliminated panel C:
//     A[i][j] <- [i not in K] A[i][j] + sum_k C[i][k] T[k][j],
// one rank-b update of the whole matrix.  In exact arithmetic this is the
// unblocked elimination; the pivots are the same (pivot = largest modulus
// among rows >= k, lowest row on ties).
constexpr int GJ_B = 32;  // panel width

// one pivot step k of the panel: pivot search in column k (rows >= k), row
// interchange and pivot-row scaling inside the panel columns, and the saved
// multipliers col[i] = A[i][k] (col[k] = 0)
__global__ __launch_bounds__(1024) void k_gjp_pivot(zd* __restrict__ A, int n, int k0, int bw, int k,
                                                    zd* __restrict__ col, int* __restrict__ perm,
                                                    int* __restrict__ flag) {
  __shared__ double bv[1024];
  __shared__ int bi[1024];
  __shared__ zd prow[GJ_B];
  const int tid = threadIdx.x;
  const int kk = k - k0;
  double best = -1.0;
  int besti = n;
  for (int i = k + tid; i < n; i += blockDim.x) {
    const double v = sqrt(norm2(A[(size_t)i * n + k]));
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
  if (tid < bw) {  // interchange rows k and p inside the panel
    const int j = k0 + tid;
    const zd ak = A[(size_t)k * n + j], ap = A[(size_t)p * n + j];
    if (p != k) A[(size_t)p * n + j] = ak;
    prow[tid] = (p != k) ? ap : ak;
  }
  __syncthreads();
  const zd piv = prow[kk];
  const double pn = norm2(piv);
  const zd inv = pn > 0 ? zd{piv.x / pn, -piv.y / pn} : zd{0, 0};
  if (tid < bw) {
    const zd a = (tid == kk) ? zd{1.0, 0.0} : prow[tid];
    A[(size_t)k * n + k0 + tid] = a * inv;
  }
  for (int i = tid; i < n; i += blockDim.x) col[i] = (i == k) ? zd{0, 0} : A[(size_t)i * n + k];
}

// eliminate column k from every other row, panel columns only
__global__ void k_gjp_elim(zd* __restrict__ A, int n, int k0, int bw, int k, const zd* __restrict__ col) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = t / GJ_B, j = t % GJ_B;
  if (i >= n || j >= bw || i == k) return;
  const int kk = k - k0;
  zd* aij = A + (size_t)i * n + k0 + j;
  const zd a = (j == kk) ? zd{0, 0} : *aij;
  *aij = a - col[i] * A[(size_t)k * n + k0 + j];
}

// the panel's row interchanges, in order, on every column outside the panel;
// then T[kk][j] = A[k0 + kk][j]
__global__ void k_gj_swap_copy(zd* __restrict__ A, int n, int k0, int bw, const int* __restrict__ perm,
                               zd* __restrict__ T) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n || (j >= k0 && j < k0 + bw)) return;
  for (int kk = 0; kk < bw; ++kk) {
    const int k = k0 + kk, p = perm[k];
    if (p != k) {
      const zd t = A[(size_t)k * n + j];
      A[(size_t)k * n + j] = A[(size_t)p * n + j];
      A[(size_t)p * n + j] = t;
    }
  }
  for (int kk = 0; kk < bw; ++kk) T[(size_t)kk * n + j] = A[(size_t)(k0 + kk) * n + j];
}

// A[i][j] = [i not in K] A[i][j] + sum_kk A[i][k0+kk] T[kk][j] for j outside the panel:
// 64 x 64 output tiles, the panel rows and the T columns of the tile in LDS
constexpr int GU_T = 64;
__global__ __launch_bounds__(256) void k_gj_update(zd* __restrict__ A, int n, int k0, int bw, const zd* __restrict__ T) {
  __shared__ zd Cs[GU_T][GJ_B + 1];
  __shared__ zd Ts[GJ_B][GU_T + 1];
  const int tid = threadIdx.x;
  const int i0 = blockIdx.y * GU_T, j0 = blockIdx.x * GU_T;
  // tiles that lie entirely inside the panel columns have nothing to do
  if (j0 >= k0 && j0 + GU_T <= k0 + bw) return;
  for (int e = tid; e < GU_T * GJ_B; e += 256) {
    const int r = e / GJ_B, c = e % GJ_B;
    Cs[r][c] = (i0 + r < n && c < bw) ? A[(size_t)(i0 + r) * n + k0 + c] : zd{0, 0};
    const int c2 = e % GU_T, r2 = e / GU_T;
    Ts[r2][c2] = (j0 + c2 < n && r2 < bw) ? T[(size_t)r2 * n + j0 + c2] : zd{0, 0};
  }
  __syncthreads();
  const int tr = tid >> 4, tc = tid & 15;  // 4 x 4 outputs: rows tr + 16 a, columns tc + 16 b
  zd acc[4][4];
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) acc[a][b] = zd{0, 0};
  for (int kk = 0; kk < bw; ++kk) {
    zd cv[4], tv[4];
    for (int a = 0; a < 4; ++a) cv[a] = Cs[tr + 16 * a][kk];
    for (int b = 0; b < 4; ++b) tv[b] = Ts[kk][tc + 16 * b];
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) acc[a][b] = acc[a][b] + cv[a] * tv[b];
  }
  for (int a = 0; a < 4; ++a) {
    const int i = i0 + tr + 16 * a;
    if (i >= n) continue;
    const bool in_panel_row = (i >= k0 && i < k0 + bw);
    for (int b = 0; b < 4; ++b) {
      const int j = j0 + tc + 16 * b;
      if (j >= n || (j >= k0 && j < k0 + bw)) continue;
      zd* aij = A + (size_t)i * n + j;
      *aij = (in_panel_row ? zd{0, 0} : *aij) + acc[a][b];
    }
  }
}

size_t gj_workspace(int n) { return (size_t)(GJ_B + 1) * n; }

void launch_gj_invert(zd* A, int n, zd* T, int* perm, int* flag, hipStream_t s) {
  zd* col = T + (size_t)GJ_B * n;
  for (int k0 = 0; k0 < n; k0 += GJ_B) {
    const int bw = (n - k0 < GJ_B) ? n - k0 : GJ_B;
    for (int k = k0; k < k0 + bw; ++k) {
      hipLaunchKernelGGL(k_gjp_pivot, dim3(1), dim3(1024), 0, s, A, n, k0, bw, k, col, perm, flag);
      hipLaunchKernelGGL(k_gjp_elim, dim3((n * GJ_B + 255) / 256), dim3(256), 0, s, A, n, k0, bw, k, col);
    }
    hipLaunchKernelGGL(k_gj_swap_copy, dim3((n + 255) / 256), dim3(256), 0, s, A, n, k0, bw, perm, T);
    hipLaunchKernelGGL(k_gj_update, dim3((n + GU_T - 1) / GU_T, (n + GU_T - 1) / GU_T), dim3(256), 0, s, A, n, k0,
                       bw, T);
  }
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

void launch_gj_unpermute(zd* A, int n, const int* perm, hipStream_t s) {
  hipLaunchKernelGGL(k_gj_unpermute, dim3((n + 63) / 64), dim3(64), 0, s, A, n, perm);
}

// y = A x, one wave per row
// V = zd, or zf for the mixed cycle: x widened exactly, y rounded to nearest
__device__ __forceinline__ zd mv_in(const zd& v) { return v; }
__device__ __forceinline__ zd mv_in(const zf& v) { return zd{(double)v.x, (double)v.y}; }
__device__ __forceinline__ void mv_out(const zd& a, zd& o) { o = a; }
__device__ __forceinline__ void mv_out(const zd& a, zf& o) { o = zf{(float)a.x, (float)a.y}; }

template <typename V>
__global__ __launch_bounds__(256) void k_dense_mv(const zd* __restrict__ A, int n, const V* __restrict__ x,
                                                  V* __restrict__ y, int nrhs) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + wave;
  if (row >= n) return;
  const zd* Ar = A + (size_t)row * n;
  for (int r = 0; r < nrhs; ++r) {
    const V* xv = x + (size_t)r * n;
    zd acc = {0, 0};
    for (int j = lane; j < n; j += 64) acc = acc + Ar[j] * mv_in(xv[j]);
    for (int off = 32; off > 0; off >>= 1) {
      acc.x += __shfl_xor(acc.x, off, 64);
      acc.y += __shfl_xor(acc.y, off, 64);
    }
    if (lane == 0) mv_out(acc, y[(size_t)r * n + row]);
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

// The FP64 product for many right-hand sides on the matrix cores
// (v_mfma_f64_16x16x4f64), the real form of k_dense_mm32: A as an n x 2n
// real matrix (re, im interleaved as stored) times the 2n x 2R matrix of
// (Re x, -Im x) / (Im x, Re x) column pairs.  A work-group owns 64 rows (16
// per wave) and 8 NT right-hand sides over one quarter of K; per 16-complex
// chunk each lane streams 4 complex entries of its row (prefetched one chunk
// ahead) and the chunk of X goes through LDS.  The partial tiles leave
// through LDS in passes of 16 right-hand sides and k_dense_mm_reduce sums
// the quarters in a fixed order, so a column's result does not depend on the
// other columns.
typedef double md4 __attribute__((ext_vector_type(4)));
// v_mfma_f64_16x16x4f64: lane l supplies A[l%16][k0 + l/16] and
// B[k0 + l/16][l%16] and receives C[l/16 + 4e][l%16], e = 0..3
static __device__ __forceinline__ md4 mfma64(double a, double b, md4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
constexpr int M64_KC = 16;
static_assert(MM_SPLIT == 4, "k_dense_mm64 writes the partials k_dense_mm_reduce sums");

template <int NT>
__global__ __launch_bounds__(256) void k_dense_mm64(const zd* __restrict__ A, int n, const zd* __restrict__ X,
                                                    zd* __restrict__ part, int nrhs, int chunks_per_split) {
  constexpr int RB = 8 * NT, XS = M64_KC + 1;
  constexpr int XPT = (RB * M64_KC + 255) / 256;
  constexpr int XBYTES = 2 * RB * XS * 16, TBYTES = 16 * 130 * 8;
  __shared__ __align__(16) char lds[XBYTES > TBYTES ? XBYTES : TBYTES];
  zd (*Xs)[RB][XS] = reinterpret_cast<zd (*)[RB][XS]>(lds);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int c = lane & 15, g = lane >> 4, q = c & 1;
  const int row0 = blockIdx.x * 64;
  const bool wave_rows = row0 + wave * 16 < n;  // n is a multiple of 16
  const int r0 = blockIdx.y * RB;
  const int nch = (n + M64_KC - 1) / M64_KC;
  const int ch0 = blockIdx.z * chunks_per_split;
  const int ch1 = min(nch, ch0 + chunks_per_split);
  const zd* Arow = A + (size_t)min(row0 + wave * 16 + c, n - 1) * n;
  md4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = md4{0.0, 0.0, 0.0, 0.0};
  zd a[4], xr[XPT];
  // chunk loads: each entry is set to zero and then loaded if in range (a
  // conditional expression between a load and a named zero makes the
  // compiler select between addresses and keep the arrays in scratch)
#define MM64_LOAD(CH)                                                                      \
  do {                                                                                     \
    _Pragma("unroll") for (int t = 0; t < 4; ++t) {                                        \
      const int k = (CH) * M64_KC + 4 * g + t;                                             \
      a[t].x = 0.0;                                                                        \
      a[t].y = 0.0;                                                                        \
      if (wave_rows && k < n) a[t] = Arow[k];                                              \
    }                                                                                      \
    _Pragma("unroll") for (int e = 0; e < XPT; ++e) {                                      \
      const int idx = tid + 256 * e, r = idx / M64_KC, k = (CH) * M64_KC + idx % M64_KC;   \
      xr[e].x = 0.0;                                                                       \
      xr[e].y = 0.0;                                                                       \
      if (idx < RB * M64_KC && r0 + r < nrhs && k < n) xr[e] = X[(size_t)(r0 + r) * n + k]; \
    }                                                                                      \
  } while (0)
  if (ch0 < ch1) MM64_LOAD(ch0);
  for (int ch = ch0; ch < ch1; ++ch) {
    const int buf = (ch - ch0) & 1;
#pragma unroll
    for (int e = 0; e < XPT; ++e) {
      const int idx = tid + 256 * e;
      if (idx < RB * M64_KC) Xs[buf][idx / M64_KC][idx % M64_KC] = xr[e];
    }
    __syncthreads();
    zd cur[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) cur[t] = a[t];
    if (ch + 1 < ch1) MM64_LOAD(ch + 1);
    // issue across the independent column-tile accumulators (each column
    // still accumulates its K-steps in the same order)
    // B entries straight from LDS at a lane-dependent offset (see k_dense_mm32)
    const double sg = q ? 1.0 : -1.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      double b0[NT], b1[NT];
#pragma unroll
      for (int ct = 0; ct < NT; ++ct) {
        // complex entry k = 4g + t of right-hand side 8 ct + c / 2
        const double* v = reinterpret_cast<const double*>(&Xs[buf][8 * ct + (c >> 1)][4 * g + t]);
        b0[ct] = v[q];
        b1[ct] = sg * v[1 - q];
      }
#pragma unroll
      for (int ct = 0; ct < NT; ++ct) acc[ct] = mfma64(cur[t].x, b0[ct], acc[ct]);
#pragma unroll
      for (int ct = 0; ct < NT; ++ct) acc[ct] = mfma64(cur[t].y, b1[ct], acc[ct]);
    }
  }
#undef MM64_LOAD
  // the 64 x RB partial tile through LDS, 16 right-hand sides (two column tiles) per pass
  double (*T)[130] = reinterpret_cast<double (*)[130]>(lds);
  zd* out = part + (size_t)blockIdx.z * nrhs * n;
#pragma unroll
  for (int h = 0; h < (NT + 1) / 2; ++h) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int ct = 2 * h + u;
      if (ct < NT) {
#pragma unroll
        for (int e = 0; e < 4; ++e) T[8 * u + (c >> 1)][2 * (wave * 16 + g + 4 * e) + q] = acc[ct][e];
      }
    }
    __syncthreads();
    for (int idx = tid; idx < 16 * 64; idx += 256) {
      const int rl = idx >> 6, i = idx & 63, rb = 16 * h + rl;
      if (rb < RB && r0 + rb < nrhs && row0 + i < n) out[(size_t)(r0 + rb) * n + row0 + i] = zd{T[rl][2 * i], T[rl][2 * i + 1]};
    }
  }
}

size_t dense_mm_workspace(int n, int nrhs) { return (size_t)MM_SPLIT * n * nrhs; }

bool launch_dense_mv_f32io(const zd* A, int n, const zf* x, zf* y, int nrhs, bool many, hipStream_t s) {
  if (many || nrhs > 2) return false;
  hipLaunchKernelGGL(k_dense_mv<zf>, dim3((n + 3) / 4), dim3(256), 0, s, A, n, x, y, nrhs);
  return true;
}

void launch_dense_mv(const zd* A, int n, const zd* x, zd* y, int nrhs, bool many, zd* work, hipStream_t s) {
  if (!many && nrhs <= 2) {
    hipLaunchKernelGGL(k_dense_mv<zd>, dim3((n + 3) / 4), dim3(256), 0, s, A, n, x, y, nrhs);
  } else if (n % 16 == 0) {
    const int nch = (n + M64_KC - 1) / M64_KC;
    const int cps = (nch + MM_SPLIT - 1) / MM_SPLIT;
    const int nt = nrhs <= 8 ? 1 : nrhs <= 16 ? 2 : nrhs <= 32 ? 4 : 8;
    const dim3 grid((n + 63) / 64, (nrhs + 8 * nt - 1) / (8 * nt), MM_SPLIT);
    switch (nt) {
      case 1: hipLaunchKernelGGL(k_dense_mm64<1>, grid, dim3(256), 0, s, A, n, x, work, nrhs, cps); break;
      case 2: hipLaunchKernelGGL(k_dense_mm64<2>, grid, dim3(256), 0, s, A, n, x, work, nrhs, cps); break;
      case 4: hipLaunchKernelGGL(k_dense_mm64<4>, grid, dim3(256), 0, s, A, n, x, work, nrhs, cps); break;
      default: hipLaunchKernelGGL(k_dense_mm64<8>, grid, dim3(256), 0, s, A, n, x, work, nrhs, cps); break;
    }
    const size_t tot = (size_t)n * nrhs;
    hipLaunchKernelGGL(k_dense_mm_reduce, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, work, n, nrhs, y);
  } else {
    hipLaunchKernelGGL(k_dense_mm, dim3((n + MM_T - 1) / MM_T, (nrhs + MM_T - 1) / MM_T, MM_SPLIT), dim3(256), 0, s,
                       A, n, x, work, nrhs);
    const size_t tot = (size_t)n * nrhs;
    hipLaunchKernelGGL(k_dense_mm_reduce, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, work, n, nrhs, y);
  }
}

// ---------------------------------------------------------------------------
// The product with half of the inverse.  The coarsest operator is
// gamma5-Hermitian, Gamma_5 D_L Gamma_5 = D_L^H (Sec. 3.5: the aggregation
// keeps the two spins apart, so every Galerkin level inherits the relation of
// the Wilson operator), and so is its inverse: A[j][i] = g_i g_j conj(A[i][j])
// with g = +1 on spin 0 and -1 on spin 1 (coarse dof 16 site + 8 s + k, so
// within a block of 64 dofs g depends on the local index alone).  The
// single-RHS product streams only the 64 x 64 blocks on and above the block
// diagonal (n^2 / 2 + 32 n entries instead of n^2): each block gives its row
// product to its own block row and its mirrored column product to the
// transposed block row.  The partial products of block row K are summed over
// the block columns in order by a second kernel (deterministic, no atomics).
// ---------------------------------------------------------------------------
constexpr int G5B = 64;
__device__ __forceinline__ double g5_local(int r) { return (r & 8) ? -1.0 : 1.0; }

// Ap[q] = block (I, J) = blk[q] of the inverse, row-major; a block off the
// diagonal holds the average of A_IJ and the mirror of A_JI (the two agree up
// to the inversion's rounding), so the packed matrix is exactly gamma5-Hermitian
template <typename S>
__global__ __launch_bounds__(256) void k_pack_g5(const zd* __restrict__ A, int n, const int* __restrict__ blk,
                                                 S* __restrict__ Ap) {
  const int q = blockIdx.x, I = blk[2 * q], J = blk[2 * q + 1];
  for (int e = threadIdx.x; e < G5B * G5B; e += 256) {
    const int r = e >> 6, c = e & 63;
    const zd a = A[(size_t)(I * G5B + r) * n + J * G5B + c];
    zd v = a;
    if (I != J) {
      const zd m = A[(size_t)(J * G5B + c) * n + I * G5B + r];
      const double g = g5_local(r) * g5_local(c);
      v = zd{0.5 * (a.x + g * m.x), 0.5 * (a.y - g * m.y)};
    }
    mv_out(v, Ap[(size_t)q * G5B * G5B + e]);  // FP32 storage: rounded to nearest
  }
}

void launch_pack_g5(const zd* A, int n, const int* blk, zd* Ap, hipStream_t s) {
  const int nbk = n / G5B;
  hipLaunchKernelGGL(k_pack_g5<zd>, dim3(nbk * (nbk + 1) / 2), dim3(256), 0, s, A, n, blk, Ap);
}
void launch_pack_g5_f32(const zd* A, int n, const int* blk, zf* Ap, hipStream_t s) {
  const int nbk = n / G5B;
  hipLaunchKernelGGL(k_pack_g5<zf>, dim3(nbk * (nbk + 1) / 2), dim3(256), 0, s, A, n, blk, Ap);
}

// a packed entry, read once per product (non-temporal), widened to FP64
__device__ __forceinline__ zd g5_load(const zd* p) {
  const double* d = reinterpret_cast<const double*>(p);
  return zd{__builtin_nontemporal_load(d), __builtin_nontemporal_load(d + 1)};
}
__device__ __forceinline__ zd g5_load(const zf* p) {
  const double w = __builtin_nontemporal_load(reinterpret_cast<const double*>(p));  // the two floats at once
  const zf v = __builtin_bit_cast(zf, w);
  return zd{(double)v.x, (double)v.y};
}

// One step of the reduce-scatter of 16 row partials over the 64 lanes: with
// mask 4 H the lane keeps the half of its 2 H rows selected by its own bit
// and adds the partner's values of the same rows
template <int H>
__device__ __forceinline__ void g5_rs_step(zd (&v)[16], int lane) {
  const bool up = (lane & (4 * H)) != 0;
#pragma unroll
  for (int k = 0; k < H; ++k) {
    const zd keep = up ? v[k + H] : v[k], send = up ? v[k] : v[k + H];
    v[k] = keep + zd{__shfl_xor(send.x, 4 * H, 64), __shfl_xor(send.y, 4 * H, 64)};
  }
}
// v[k]: the lane's partial of row k (k = 0..15); returns in lane l the full
// sum of row l >> 2 (the 4 lanes of a quad hold the same value)
__device__ __forceinline__ zd g5_rowsum(zd (&v)[16], int lane) {
  g5_rs_step<8>(v, lane);
  g5_rs_step<4>(v, lane);
  g5_rs_step<2>(v, lane);
  g5_rs_step<1>(v, lane);
  zd rs = v[0];
  rs = rs + zd{__shfl_xor(rs.x, 2, 64), __shfl_xor(rs.y, 2, 64)};
  return rs + zd{__shfl_xor(rs.x, 1, 64), __shfl_xor(rs.y, 1, 64)};
}

// One work-group per packed block: wave w holds rows w, w + 4, ..., w + 60,
// lane c column c.  x_I and x_J go through LDS.  The column products come
// first (sums along each lane's rows, then over the four waves in order
// through LDS); the row products are then formed in place over the block's
// registers and summed by a reduce-scatter over the lanes (xor 32, 16, 8, 4
// halve the rows each lane carries, xor 2 and 1 finish), which keeps the
// register count low enough for 5 work-groups per CU.
// part[((r nbk + K) nbk + L) 64 + i]: block (K, L)'s contribution to y_r.
template <typename S, typename V, int NR>
__global__ __launch_bounds__(256) void k_dense_mv_g5(const S* __restrict__ Ap, const int* __restrict__ blk, int nbk,
                                                     int n, const V* __restrict__ x, zd* __restrict__ part) {
  __shared__ zd xsh[NR][2][G5B];  // [r][0]: x_I, [r][1]: x_J
  __shared__ zd colsh[NR][4][G5B];
  const int q = blockIdx.x, I = blk[2 * q], J = blk[2 * q + 1];
  // the wave index is uniform over the wave: the x_I values of its rows are
  // then scalar operands, not registers per lane
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const S* B = Ap + (size_t)q * G5B * G5B + (size_t)wave * G5B + lane;
  zd a[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) a[k] = g5_load(B + (size_t)k * 4 * G5B);
  if (threadIdx.x < NR * 2 * G5B) {
    const int r = threadIdx.x / (2 * G5B), h = (threadIdx.x / G5B) & 1;
    xsh[r][h][lane] = mv_in(x[(size_t)r * n + (h ? J : I) * G5B + lane]);
  }
  __syncthreads();
  if (I != J) {  // uniform over the work-group
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      zd cs = {0, 0};
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int row = wave + 4 * k;
        const zd t = cjmul(a[k], xsh[r][0][row]);
        cs = cs + zd{g5_local(row) * t.x, g5_local(row) * t.y};
      }
      colsh[r][wave][lane] = cs;
    }
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const zd xj = xsh[r][1][lane];
    zd rs;
    if (r == NR - 1) {  // the block's last use: in place
#pragma unroll
      for (int k = 0; k < 16; ++k) a[k] = a[k] * xj;
      rs = g5_rowsum(a, lane);
    } else {
      zd v[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) v[k] = a[k] * xj;
      rs = g5_rowsum(v, lane);
    }
    if ((lane & 3) == 0) part[(((size_t)r * nbk + I) * nbk + J) * G5B + wave + 4 * (lane >> 2)] = rs;
  }
  if (I == J) return;  // uniform over the work-group
  __syncthreads();
  if (wave < NR) {
    const zd c = ((colsh[wave][0][lane] + colsh[wave][1][lane]) + colsh[wave][2][lane]) + colsh[wave][3][lane];
    const double g = g5_local(lane);
    part[(((size_t)wave * nbk + J) * nbk + I) * G5B + lane] = zd{g * c.x, g * c.y};
  }
}

// y_r[K 64 + e] = sum over the block columns L of part[r][K][L][e]: one
// work-group per (K, r); thread group g (of 8) sums L = g, g + 8, ... in
// order, then the 8 partial sums are added in order
template <typename V>
__global__ __launch_bounds__(512) void k_dense_mv_g5_reduce(const zd* __restrict__ part, int nbk, int n,
                                                            V* __restrict__ y) {
  __shared__ zd sh[8][G5B];
  const int K = blockIdx.x, r = blockIdx.y, e = threadIdx.x & 63, g = threadIdx.x >> 6;
  const zd* p = part + (((size_t)r * nbk + K) * nbk) * G5B + e;
  zd acc = {0, 0};
#pragma unroll 4
  for (int L = g; L < nbk; L += 8) acc = acc + p[(size_t)L * G5B];
  sh[g][e] = acc;
  __syncthreads();
  if (g == 0) {
    zd t = sh[0][e];
#pragma unroll
    for (int k = 1; k < 8; ++k) t = t + sh[k][e];
    mv_out(t, y[(size_t)r * n + K * G5B + e]);
  }
}

template <typename S, typename V>
static bool dense_mv_g5(const S* Ap, const int* blk, int n, const V* x, V* y, int nrhs, zd* part, hipStream_t s) {
  if (!Ap || nrhs < 1 || nrhs > 2 || n % G5B != 0) return false;
  const int nbk = n / G5B, nblk = nbk * (nbk + 1) / 2;
  if (nrhs == 1)
    hipLaunchKernelGGL((k_dense_mv_g5<S, V, 1>), dim3(nblk), dim3(256), 0, s, Ap, blk, nbk, n, x, part);
  else
    hipLaunchKernelGGL((k_dense_mv_g5<S, V, 2>), dim3(nblk), dim3(256), 0, s, Ap, blk, nbk, n, x, part);
  hipLaunchKernelGGL(k_dense_mv_g5_reduce<V>, dim3(nbk, nrhs), dim3(512), 0, s, part, nbk, n, y);
  return true;
}

bool launch_dense_mv_g5(const zd* Ap, const int* blk, int n, const zd* x, zd* y, int nrhs, zd* part, hipStream_t s) {
  return dense_mv_g5(Ap, blk, n, x, y, nrhs, part, s);
}
bool launch_dense_mv_g5_f32io(const zd* Ap, const int* blk, int n, const zf* x, zf* y, int nrhs, zd* part,
                              hipStream_t s) {
  return dense_mv_g5(Ap, blk, n, x, y, nrhs, part, s);
}
bool launch_dense_mv_g5_c32(const zf* Ap, const int* blk, int n, const zf* x, zf* y, int nrhs, zd* part,
                            hipStream_t s) {
  return dense_mv_g5(Ap, blk, n, x, y, nrhs, part, s);
}

// ---------------------------------------------------------------------------
// The coarsest solve of the mixed-precision cycle: the cycle's coarse
// correction is FP32 in and out, and the inverse is read from an FP32 copy
// (rounded to nearest from the FP64 inverse), which halves the bytes of the
// dominant read.
// ---------------------------------------------------------------------------

// y = A x for NR = 1 or 2 right-hand sides: one wave per row, two complex
// entries per 16-byte load, products and sums in FP64, the row of A read once
// for both right-hand sides.  n is a multiple of 16.
template <int NR>
__global__ __launch_bounds__(256) void k_dense_mv32(const zf* __restrict__ A, int n, const zf* __restrict__ x,
                                                    zf* __restrict__ y) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + wave;
  if (row >= n) return;
  const float4* Ar = reinterpret_cast<const float4*>(A + (size_t)row * n);
  const int n2 = n >> 1;
  double re[NR], im[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) re[r] = im[r] = 0.0;
#pragma unroll 4
  for (int j = lane; j < n2; j += 64) {
    const float4 a = Ar[j];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const float4 v = reinterpret_cast<const float4*>(x + (size_t)r * n)[j];
      re[r] += (double)a.x * v.x - (double)a.y * v.y + (double)a.z * v.z - (double)a.w * v.w;
      im[r] += (double)a.x * v.y + (double)a.y * v.x + (double)a.z * v.w + (double)a.w * v.z;
    }
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    for (int off = 32; off > 0; off >>= 1) {
      re[r] += __shfl_xor(re[r], off, 64);
      im[r] += __shfl_xor(im[r], off, 64);
    }
    if (lane == 0) y[(size_t)r * n + row] = zf{(float)re[r], (float)im[r]};
  }
}

// Y = A X for many right-hand sides on the matrix cores.  The complex product
// is the real product of A viewed as an n x 2n real matrix (re, im
// interleaved, as stored) with the 2n x 2R real matrix whose column pair for
// right-hand side r holds (Re x, -Im x) and (Im x, Re x) interleaved along K:
// column 2r gives Re y_r and column 2r+1 gives Im y_r.  A work-group owns 64
// rows (16 per wave) and 8 NT right-hand sides over one K slice (split-K);
// each lane streams 8 complex entries of its row per 32-complex chunk (four
// 16-byte loads, prefetched one chunk ahead), the chunk of X goes through LDS.
// Every output element sums its K range in a fixed order that does not depend
// on the other columns, so a column's result does not depend on the batch.
constexpr int M32_KC = 32, M32_SPLIT = 8;

typedef float mf4 __attribute__((ext_vector_type(4)));
// v_mfma_f32_16x16x4f32: lane l supplies A[l%16][k0 + l/16] and
// B[k0 + l/16][l%16] and receives C[4(l/16) + e][l%16], e = 0..3
static __device__ __forceinline__ mf4 mfma4(float a, float b, mf4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int NT>
__global__ __launch_bounds__(256) void k_dense_mm32(const zf* __restrict__ A, int n, const zf* __restrict__ X,
                                                    zf* __restrict__ part, int nrhs, int chunks_per_split) {
  constexpr int RB = 8 * NT;            // right-hand sides of the work-group
  constexpr int XQ = M32_KC / 2;        // float4 (two complex) per right-hand side and chunk
  constexpr int XS = XQ + 1;            // padded LDS row
  constexpr int XPT = (RB * XQ + 255) / 256;
  constexpr int XBYTES = 2 * RB * XS * 16, TBYTES = RB * 64 * 8;
  __shared__ __align__(16) char lds[XBYTES > TBYTES ? XBYTES : TBYTES];
  float4 (*Xs)[RB][XS] = reinterpret_cast<float4 (*)[RB][XS]>(lds);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int c = lane & 15, g = lane >> 4, q = c & 1;
  const int row0 = blockIdx.x * 64;
  const bool wave_rows = row0 + wave * 16 < n;  // n is a multiple of 16
  const int r0 = blockIdx.y * RB;
  const int nch = (n + M32_KC - 1) / M32_KC;
  const int ch0 = blockIdx.z * chunks_per_split;
  const int ch1 = min(nch, ch0 + chunks_per_split);
  const float4* Arow = reinterpret_cast<const float4*>(A + (size_t)min(row0 + wave * 16 + c, n - 1) * n);
  mf4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = mf4{0.f, 0.f, 0.f, 0.f};
  float4 a[4], xr[XPT];
  // chunk loads: each entry is set to zero and then loaded if in range (a
  // conditional expression between a load and a named zero makes the
  // compiler select between addresses and keep the arrays in scratch)
#define MM32_LOAD(CH)                                                                      \
  do {                                                                                     \
    _Pragma("unroll") for (int t = 0; t < 4; ++t) {                                        \
      const int k = (CH) * M32_KC + 8 * g + 2 * t; /* complex column of the pair */        \
      a[t] = make_float4(0.f, 0.f, 0.f, 0.f);                                              \
      if (wave_rows && k < n) a[t] = Arow[k >> 1];                                         \
    }                                                                                      \
    _Pragma("unroll") for (int e = 0; e < XPT; ++e) {                                      \
      const int idx = tid + 256 * e, r = idx / XQ, k = (CH) * M32_KC + 2 * (idx % XQ);     \
      xr[e] = make_float4(0.f, 0.f, 0.f, 0.f);                                             \
      if (idx < RB * XQ && r0 + r < nrhs && k < n)                                         \
        xr[e] = reinterpret_cast<const float4*>(X + (size_t)(r0 + r) * n)[k >> 1];         \
    }                                                                                      \
  } while (0)
  if (ch0 < ch1) MM32_LOAD(ch0);
  for (int ch = ch0; ch < ch1; ++ch) {
    const int buf = (ch - ch0) & 1;
#pragma unroll
    for (int e = 0; e < XPT; ++e) {
      const int idx = tid + 256 * e;
      if (idx < RB * XQ) Xs[buf][idx / XQ][idx % XQ] = xr[e];
    }
    __syncthreads();
    float4 cur[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) cur[t] = a[t];
    if (ch + 1 < ch1) MM32_LOAD(ch + 1);
    // the column tiles' accumulators are independent: issue across them so
    // that consecutive MFMAs do not wait on each other (each column still
    // accumulates its K-steps in the same order)
    // B entries straight from LDS at a lane-dependent offset: for the pair
    // (Re x_k, Im x_k) the column 2r takes (Re, -Im) and 2r+1 takes (Im, Re)
    const float sg = q ? 1.f : -1.f;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      float b0[NT], b1[NT], b2[NT], b3[NT];
#pragma unroll
      for (int ct = 0; ct < NT; ++ct) {
        // complex entries k = 8g + 2t and k + 1 of right-hand side 8 ct + c / 2
        const float* v = reinterpret_cast<const float*>(&Xs[buf][8 * ct + (c >> 1)][4 * g + t]);
        b0[ct] = v[q];
        b1[ct] = sg * v[1 - q];
        b2[ct] = v[2 + q];
        b3[ct] = sg * v[3 - q];
      }
#pragma unroll
      for (int ct = 0; ct < NT; ++ct) acc[ct] = mfma4(cur[t].x, b0[ct], acc[ct]);
#pragma unroll
      for (int ct = 0; ct < NT; ++ct) acc[ct] = mfma4(cur[t].y, b1[ct], acc[ct]);
#pragma unroll
      for (int ct = 0; ct < NT; ++ct) acc[ct] = mfma4(cur[t].z, b2[ct], acc[ct]);
#pragma unroll
      for (int ct = 0; ct < NT; ++ct) acc[ct] = mfma4(cur[t].w, b3[ct], acc[ct]);
    }
  }
#undef MM32_LOAD
  // transpose the 64 x RB tile through LDS so that the partials are written
  // along the rows of each right-hand side
  __syncthreads();
  float (*T)[130] = reinterpret_cast<float (*)[130]>(lds);
  static_assert(RB * 130 * 4 <= (XBYTES > TBYTES ? XBYTES : TBYTES), "transpose tile exceeds LDS");
#pragma unroll
  for (int ct = 0; ct < NT; ++ct)
#pragma unroll
    for (int e = 0; e < 4; ++e) T[8 * ct + (c >> 1)][2 * (wave * 16 + 4 * g + e) + q] = acc[ct][e];
  __syncthreads();
  zf* out = part + (size_t)blockIdx.z * nrhs * n;
  for (int idx = tid; idx < RB * 64; idx += 256) {
    const int r = idx >> 6, i = idx & 63;
    if (r0 + r < nrhs && row0 + i < n) out[(size_t)(r0 + r) * n + row0 + i] = zf{T[r][2 * i], T[r][2 * i + 1]};
  }
}

__global__ void k_dense_mm32_reduce(const zf* __restrict__ part, size_t tot, zf* __restrict__ Y) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= tot) return;
  zf s = part[t];
#pragma unroll
  for (int q = 1; q < M32_SPLIT; ++q) s = s + part[(size_t)q * tot + t];
  Y[t] = s;
}

size_t dense_mm32_workspace_bytes(int n, int nrhs) { return (size_t)M32_SPLIT * n * nrhs * sizeof(zf); }

void launch_dense_mv32(const zf* A, int n, const zf* x, zf* y, int nrhs, bool many, zf* work, hipStream_t s) {
  if (!many && nrhs <= 2) {
    if (nrhs == 1) hipLaunchKernelGGL(k_dense_mv32<1>, dim3((n + 3) / 4), dim3(256), 0, s, A, n, x, y);
    else hipLaunchKernelGGL(k_dense_mv32<2>, dim3((n + 3) / 4), dim3(256), 0, s, A, n, x, y);
    return;
  }
  const int nch = (n + M32_KC - 1) / M32_KC;
  const int cps = (nch + M32_SPLIT - 1) / M32_SPLIT;
  const int nt = nrhs <= 8 ? 1 : nrhs <= 16 ? 2 : nrhs <= 32 ? 4 : 8;
  const dim3 grid((n + 63) / 64, (nrhs + 8 * nt - 1) / (8 * nt), M32_SPLIT);
  switch (nt) {
    case 1: hipLaunchKernelGGL(k_dense_mm32<1>, grid, dim3(256), 0, s, A, n, x, work, nrhs, cps); break;
    case 2: hipLaunchKernelGGL(k_dense_mm32<2>, grid, dim3(256), 0, s, A, n, x, work, nrhs, cps); break;
    case 4: hipLaunchKernelGGL(k_dense_mm32<4>, grid, dim3(256), 0, s, A, n, x, work, nrhs, cps); break;
    default: hipLaunchKernelGGL(k_dense_mm32<8>, grid, dim3(256), 0, s, A, n, x, work, nrhs, cps); break;
  }
  const size_t tot = (size_t)n * nrhs;
  hipLaunchKernelGGL(k_dense_mm32_reduce, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, work, tot, y);
}

}  // namespace bamg
