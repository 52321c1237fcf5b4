// Kernels of the bootstrap multigrid eigensolver (Sec. 3.4; Theorem 1 of
// Sec. 3.5).  With R = (Gamma_5 P)^H and P orthonormal per aggregate the mass
// matrices are T_l = Q_l = I, and the singular-triplet systems become the
// Hermitian eigenproblem Z_l v = lambda v, Z_l = Gamma_5 D_l.  Gamma_5 is +1 on
// spin 0 and -1 on spin 1: fine dof 2 site + s, coarse dof 16 site + 8 s + k.
//  - Ritz values lambda = <Z v, v> / <v, v> (eq. eqevZ with T = I);
//  - Kaczmarz on (D_l - lambda Gamma_5) v = 0 on coarse levels (the fine level
//    uses k_kaczmarz_fine with a shift);
//  - the least squares fit of P with more test vectors than coarse columns:
//    the best rank-8 fit per aggregate and spin (the 8 dominant eigenvectors
//    of B B^H by cyclic Jacobi rotations), with the basis fixed as the
//    Gram-Schmidt basis of the projected first 8 test vectors;
//  - Gamma_5 scaling and block combinations for the coarsest eigensolver.
#include "bamg_internal.h"

namespace bamg {

constexpr int BTR = 256;

__device__ __forceinline__ double g5_of(size_t i, int dps) {
  const int s = (dps == 2) ? (int)(i & 1) : (int)((i & 15) >> 3);
  return s ? -1.0 : 1.0;
}

// ---------------------------------------------------------------------------
// Ritz values: partial sums per block of conj(v) g5 (A v) and |v|^2, then
// lambda_r = Re(num) / den (fixed block decomposition, deterministic)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BTR) void k_ritz_partial(const zd* __restrict__ V, const zd* __restrict__ AV, size_t n,
                                                      int dps, zd* __restrict__ partial) {
  __shared__ zd sh[BTR];
  const int b = blockIdx.x, r = blockIdx.y, nb = gridDim.x;
  const size_t chunk = (n + nb - 1) / nb;
  const size_t lo = (size_t)b * chunk, hi = (lo + chunk < n) ? lo + chunk : n;
  const zd* v = V + (size_t)r * n;
  const zd* av = AV + (size_t)r * n;
  zd acc = {0, 0};  // (Re num, den)
  for (size_t i = lo + threadIdx.x; i < hi; i += BTR) {
    acc.x += g5_of(i, dps) * cjmul(v[i], av[i]).x;
    acc.y += norm2(v[i]);
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int off = BTR / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) sh[threadIdx.x] = sh[threadIdx.x] + sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(size_t)r * nb + b] = sh[0];
}

__global__ __launch_bounds__(BTR) void k_ritz_final(const zd* __restrict__ partial, int nb, double* __restrict__ lam) {
  __shared__ zd sh[BTR];
  const int r = blockIdx.x;
  zd acc = {0, 0};
  for (int b = threadIdx.x; b < nb; b += BTR) acc = acc + partial[(size_t)r * nb + b];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int off = BTR / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) sh[threadIdx.x] = sh[threadIdx.x] + sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) lam[r] = sh[0].y > 0 ? sh[0].x / sh[0].y : 0.0;
}

void launch_ritz(const zd* V, const zd* AV, size_t n, int dps, int k, zd* partial, double* lam, hipStream_t s) {
  const int nb = blas_nblocks(n);
  hipLaunchKernelGGL(k_ritz_partial, dim3(nb, k), dim3(BTR), 0, s, V, AV, n, dps, partial);
  hipLaunchKernelGGL(k_ritz_final, dim3(k), dim3(BTR), 0, s, partial, nb, lam);
}

// y_r = Gamma_5 x_r
__global__ void k_gamma5(const zd* __restrict__ x, zd* __restrict__ y, size_t n, int dps) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (i < n) y[(size_t)r * n + i] = g5_of(i, dps) * x[(size_t)r * n + i];
}

void launch_gamma5(const zd* x, zd* y, size_t n, int dps, int k, hipStream_t s) {
  hipLaunchKernelGGL(k_gamma5, dim3((unsigned)((n + 255) / 256), k), dim3(256), 0, s, x, y, n, dps);
}

// Y_j = sum_i X_i C[i][j] for p vectors of length n (C p x p row-major, device)
__global__ void k_block_combine(const zd* __restrict__ X, const zd* __restrict__ C, zd* __restrict__ Y, size_t n,
                                int p) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (t >= n) return;
  zd acc = {0, 0};
  for (int i = 0; i < p; ++i) acc = acc + X[(size_t)i * n + t] * C[(size_t)i * p + j];
  Y[(size_t)j * n + t] = acc;
}

void launch_block_combine(const zd* X, const zd* C, zd* Y, size_t n, int p, hipStream_t s) {
  hipLaunchKernelGGL(k_block_combine, dim3((unsigned)((n + 255) / 256), p), dim3(256), 0, s, X, C, Y, n, p);
}

// R_j = A_j - lam_j B_j (lam on the device)
__global__ void k_eig_residual(const zd* __restrict__ A, const zd* __restrict__ B, const double* __restrict__ lam,
                               zd* __restrict__ R, size_t n) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (t < n) R[(size_t)j * n + t] = A[(size_t)j * n + t] - lam[j] * B[(size_t)j * n + t];
}

void launch_eig_residual(const zd* A, const zd* B, const double* lam, zd* R, size_t n, int k, hipStream_t s) {
  hipLaunchKernelGGL(k_eig_residual, dim3((unsigned)((n + 255) / 256), k), dim3(256), 0, s, A, B, lam, R, n);
}

// ---------------------------------------------------------------------------
// Kaczmarz on (D_l - lambda_r Gamma_5) x_r = 0, coarse level, one colour: one
// work-group per (site, vector); the 16 rows of the site are projected in
// order, thread t < 112 owning the unknown (offset t / 16, dof t % 16) of the
// row support.  Supports of one colour are disjoint (the extents are >= 4 on
// every smoothed level, so no two offsets reach the same site).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int cwrap_b(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

__device__ __forceinline__ int colour_site_b(int c, int mode, int t, int ex) {
  if (mode == 8) {
    const int per = ex >> 3, ay = t / per;
    return ay * ex + 8 * (t - ay * per) + ((c + 3 * ay) & 7);
  }
  if (mode == 16) {
    const int per = ex >> 2, r = t / per;
    return (4 * r + (c >> 2)) * ex + 4 * (t - r * per) + (c & 3);
  }
  return c;
}

__global__ __launch_bounds__(128) void k_kaczmarz_coarse_shift(Coarse c, int colour, int mode, zd* __restrict__ x,
                                                               const double* __restrict__ lam) {
  constexpr int odx[NOFF] = {0, 1, -1, 0, 0, 1, -1};
  constexpr int ody[NOFF] = {0, 0, 0, 1, -1, 1, -1};
  __shared__ zd red[2];
  __shared__ double nred[2];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int site = colour_site_b(colour, mode, blockIdx.x, c.ex);
  const int ax = site % c.ex, ay = site / c.ex;
  const size_t n = (size_t)c.ex * c.ey * 16;
  zd* xv = x + (size_t)blockIdx.y * n;
  const double l = lam[blockIdx.y];
  const bool act = tid < NOFF * 16;
  const int o = act ? tid >> 4 : 0, j = tid & 15;
  const int nbs = cwrap_b(ay + ody[o], c.ey) * c.ex + cwrap_b(ax + odx[o], c.ex);
  zd xj = act ? xv[(size_t)nbs * 16 + j] : zd{0, 0};
  for (int i = 0; i < 16; ++i) {
    zd a = act ? c.D[(((size_t)site * NOFF + o) * 16 + i) * 16 + j] : zd{0, 0};
    if (act && o == 0 && j == i) a.x -= l * (i < 8 ? 1.0 : -1.0);
    zd rp = act ? a * xj : zd{0, 0};
    double np = norm2(a);
    for (int off = 32; off > 0; off >>= 1) {
      rp.x += __shfl_xor(rp.x, off, 64);
      rp.y += __shfl_xor(rp.y, off, 64);
      np += __shfl_xor(np, off, 64);
    }
    if (lane == 0) {
      red[wv] = rp;
      nred[wv] = np;
    }
    __syncthreads();
    const zd res = zd{0, 0} - (red[0] + red[1]);
    const double nu = nred[0] + nred[1];
    __syncthreads();
    if (nu > 0 && act) xj = xj + cdiv_real(res, nu) * conj(a);
  }
  if (act) xv[(size_t)nbs * 16 + j] = xj;
}

void launch_kaczmarz_coarse_shift(const Coarse& c, int colour, int mode, int nsites, zd* x, const double* lam,
                                  int nrhs, hipStream_t s) {
  hipLaunchKernelGGL(k_kaczmarz_coarse_shift, dim3(nsites, nrhs), dim3(128), 0, s, c, colour, mode, x, lam);
}

// ---------------------------------------------------------------------------
// Least squares fit with k (8 < k <= 16) test vectors: one work-group per
// (aggregate, spin) block of R rows (16 on level 0, 32 above).
// ---------------------------------------------------------------------------
constexpr int FK = 16;  // test vectors at most
constexpr int FR = 32;  // rows at most

// dof of row r of block (a, s): level 0 uses the 4 x 4 even-site aggregates of
// the half-x grid (row 4 (y mod 4) + (xh mod 4)), coarse levels the 2 x 2 site
// aggregates (row 8 * local site + k, local site 2 (ay mod 2) + (ax mod 2))
__device__ __forceinline__ size_t fit_dof(bool fine, int ex, int a, int s, int r) {
  if (fine) {  // ex = NH (half-x extent)
    const int cxn = ex / 4, Ax = a % cxn, Ay = a / cxn;
    const int e = (4 * Ay + (r >> 2)) * ex + 4 * Ax + (r & 3);
    return (size_t)2 * e + s;
  }
  const int cex = ex / 2, AX = a % cex, AY = a / cex;
  const int t = r >> 3, k = r & 7;
  const int site = (2 * AY + (t >> 1)) * ex + 2 * AX + (t & 1);
  return (size_t)site * 16 + 8 * s + k;
}

__global__ __launch_bounds__(64) void k_fit_ls(bool fine, int ex, int R, size_t n, const zd* __restrict__ V, int k,
                                               zd* __restrict__ P) {
  __shared__ zd B[FR][FK];
  __shared__ zd H[FR][FR + 1];
  __shared__ zd E[FR][FR + 1];
  __shared__ zd W[FR][8];
  __shared__ zd Cc[8][8];
  __shared__ double wdiag[FR];
  __shared__ int idx[8];
  __shared__ zd rot[4];  // U_pp, U_pq, U_qp, U_qq
  __shared__ int skip;
  __shared__ double offn, fro;
  const int tid = threadIdx.x;
  const int a = blockIdx.x >> 1, s = blockIdx.x & 1;
  for (int e = tid; e < R * k; e += 64) {
    const int r = e / k, j = e % k;
    B[r][j] = V[(size_t)j * n + fit_dof(fine, ex, a, s, r)];
  }
  __syncthreads();
  // H = B B^H, E = I
  for (int e = tid; e < R * R; e += 64) {
    const int i = e / R, i2 = e % R;
    zd acc = {0, 0};
    for (int j = 0; j < k; ++j) acc = acc + B[i][j] * conj(B[i2][j]);
    H[i][i2] = acc;
    E[i][i2] = zd{i == i2 ? 1.0 : 0.0, 0.0};
  }
  __syncthreads();
  if (tid == 0) {
    double f = 0;
    for (int i = 0; i < R; ++i)
      for (int i2 = 0; i2 < R; ++i2) f += norm2(H[i][i2]);
    fro = f;
  }
  __syncthreads();
  for (int sweep = 0; sweep < 100; ++sweep) {
    if (tid == 0) {
      double off = 0;
      for (int i = 0; i < R; ++i)
        for (int i2 = 0; i2 < R; ++i2)
          if (i != i2) off += norm2(H[i][i2]);
      offn = off;
    }
    __syncthreads();
    if (offn <= 1e-30 * fro || offn == 0.0) break;
    for (int p = 0; p < R - 1; ++p)
      for (int q = p + 1; q < R; ++q) {
        if (tid == 0) {
          const zd hpq = H[p][q];
          const double r = sqrt(norm2(hpq));
          skip = (r == 0.0);
          if (r != 0.0) {
            const zd ph = cdiv_real(hpq, r);
            const double aa = H[p][p].x, bb = H[q][q].x;
            const double tau = (bb - aa) / (2.0 * r);
            const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            const double cc = 1.0 / sqrt(1.0 + t * t), sn = t * cc;
            rot[0] = zd{cc, 0.0};
            rot[1] = zd{sn, 0.0};
            rot[2] = (-sn) * conj(ph);
            rot[3] = cc * conj(ph);
          }
        }
        __syncthreads();
        if (!skip) {
          const zd upp = rot[0], upq = rot[1], uqp = rot[2], uqq = rot[3];
          if (tid < R) {  // H <- H U (columns p, q)
            const zd hkp = H[tid][p], hkq = H[tid][q];
            H[tid][p] = hkp * upp + hkq * uqp;
            H[tid][q] = hkp * upq + hkq * uqq;
          }
          __syncthreads();
          if (tid < R) {  // H <- U^H H (rows p, q)
            const zd hpk = H[p][tid], hqk = H[q][tid];
            H[p][tid] = conj(upp) * hpk + conj(uqp) * hqk;
            H[q][tid] = conj(upq) * hpk + conj(uqq) * hqk;
          } else if (tid >= 32 && tid - 32 < R) {  // E <- E U
            const int kk = tid - 32;
            const zd ekp = E[kk][p], ekq = E[kk][q];
            E[kk][p] = ekp * upp + ekq * uqp;
            E[kk][q] = ekp * upq + ekq * uqq;
          }
          __syncthreads();
          if (tid == 0) {
            H[p][q] = zd{0, 0};
            H[q][p] = zd{0, 0};
            H[p][p].y = 0.0;
            H[q][q].y = 0.0;
          }
        }
        __syncthreads();
      }
  }
  // the 8 largest eigenvalues (ties: lowest index)
  if (tid < R) wdiag[tid] = H[tid][tid].x;
  __syncthreads();
  if (tid == 0) {
    unsigned long long used = 0;
    for (int e = 0; e < 8; ++e) {
      int best = -1;
      for (int i = 0; i < R; ++i)
        if (!((used >> i) & 1ull) && (best < 0 || wdiag[i] > wdiag[best])) best = i;
      idx[e] = best;
      used |= 1ull << best;
    }
  }
  __syncthreads();
  // coefficients of the first 8 test vectors on the 8 eigenvectors, then projections
  {
    const int e = tid >> 3, j = tid & 7;  // 64 threads = 8 x 8
    zd acc = {0, 0};
    for (int i = 0; i < R; ++i) acc = acc + cjmul(E[i][idx[e]], B[i][j]);
    Cc[e][j] = acc;
  }
  __syncthreads();
  if (tid < R)
    for (int j = 0; j < 8; ++j) {
      zd acc = {0, 0};
      for (int e = 0; e < 8; ++e) acc = acc + E[tid][idx[e]] * Cc[e][j];
      W[tid][j] = acc;
    }
  __syncthreads();
  // Gram-Schmidt (applied twice, R_jj > 0) in column order
  if (tid == 0) {
    for (int j = 0; j < 8; ++j) {
      for (int pass = 0; pass < 2; ++pass) {
        zd hq[8];
        for (int q = 0; q < j; ++q) {
          zd acc = {0, 0};
          for (int i = 0; i < R; ++i) acc = acc + cjmul(W[i][q], W[i][j]);
          hq[q] = acc;
        }
        for (int q = 0; q < j; ++q)
          for (int i = 0; i < R; ++i) W[i][j] = W[i][j] - W[i][q] * hq[q];
      }
      double nrm = 0;
      for (int i = 0; i < R; ++i) nrm += norm2(W[i][j]);
      nrm = sqrt(nrm);
      for (int i = 0; i < R; ++i) W[i][j] = nrm > 0 ? cdiv_real(W[i][j], nrm) : zd{0, 0};
    }
  }
  __syncthreads();
  for (int e = tid; e < R * 8; e += 64) {
    const int r = e >> 3, j = e & 7;
    P[(((size_t)a * 2 + s) * R + r) * 8 + j] = W[r][j];
  }
}

void launch_fit_ls(bool fine, int ex, int ey, const zd* V, int k, zd* P, hipStream_t s) {
  // fine: ex = NH, ey = N; blocks of 16 rows; coarse: ex x ey sites, blocks of 32 rows
  const int R = fine ? 16 : 32;
  const int nagg = fine ? (ex / 4) * (ey / 4) : (ex / 2) * (ey / 2);
  const size_t n = fine ? (size_t)ex * ey * 2 : (size_t)ex * ey * 16;
  hipLaunchKernelGGL(k_fit_ls, dim3(nagg * 2), dim3(64), 0, s, fine, ex, R, n, V, k, P);
}

}  // namespace bamg
