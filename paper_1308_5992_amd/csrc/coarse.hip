// Coarse-level kernels: the Galerkin block stencil D_l (16 x 16 complex blocks
// on the 7 offsets that the 4x4-then-2x2 aggregation of the odd-even reduced
// operator produces, Sec. 3.2 / 3.5), its multicolour Kaczmarz smoother
// (Sec. 3.1), the 2x2 aggregate transfers and least-squares fit (Sec. 3.3),
// the Galerkin product of the next level and the dense expansion of the
// coarsest operator.
//
// A wave (64 lanes) owns one coarse site: lane = 4*i + q holds row i of the
// site's 16 x 112 block row, columns 4q..4q+3 of each of the 7 blocks.
#include "bamg_internal.h"

namespace bamg {

__device__ __forceinline__ int cwrap(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

__constant__ int ODX[NOFF] = {0, 1, -1, 0, 0, 1, -1};
__constant__ int ODY[NOFF] = {0, 0, 0, 1, -1, 1, -1};

__device__ __forceinline__ int coarse_offset_index(int dx, int dy) {
  for (int o = 0; o < NOFF; ++o)
    if (ODX[o] == dx && ODY[o] == dy) return o;
  return -1;
}

__device__ __forceinline__ int neighbour_site(int site, int o, int ex, int ey) {
  const int ax = site % ex, ay = site / ex;
  return cwrap(ay + ODY[o], ey) * ex + cwrap(ax + ODX[o], ex);
}

template <typename T>
__device__ __forceinline__ cx<T> shfl_xor_z(cx<T> v, int m) {
  return cx<T>{__shfl_xor(v.x, m, 64), __shfl_xor(v.y, m, 64)};
}

// the value of lane i ^ M (M = 1, 2, 4) by DPP moves: quad permutations for 1
// and 2; for 4, a row shift down for lanes with bit 2 set, up for the others
template <int M, typename R>
__device__ __forceinline__ R dpp_xor(R v) {
  if constexpr (M == 1) {
    return dpp_mov<DPP_QUAD_XOR1>(v);
  } else if constexpr (M == 2) {
    return dpp_mov<DPP_QUAD_XOR2>(v);
  } else {
    static_assert(M == 4, "lane masks 1, 2, 4");
    const R dn = dpp_mov<DPP_ROW_SHR4>(v), up = dpp_mov<DPP_ROW_SHL4>(v);
    return (threadIdx.x & 4) ? dn : up;
  }
}
template <int M, typename T>
__device__ __forceinline__ cx<T> xor_add(cx<T> v) {
  return cx<T>{v.x + dpp_xor<M>(v.x), v.y + dpp_xor<M>(v.y)};
}

// ---------------------------------------------------------------------------
// y = D x  (or y = b - D x)
// ---------------------------------------------------------------------------
// A wave's share of (D x)_site: lane 4 i + q loads row i, columns 4q..4q+3 of
// each of the 7 blocks (and the neighbour sites), then coarse_apply_row sums
// them against x in a fixed order and over the quad.  k_coarse_apply and the
// fused residual-restriction kernel call both, so they give the same bits.
template <typename T, typename S>
__device__ __forceinline__ void coarse_apply_load(const CoarseT<T, S>& c, int site, int i, int q, cx<T> (&Dv)[NOFF][4],
                                                  int (&nb)[NOFF]) {
  for (int o = 0; o < NOFF; ++o) {
    nb[o] = neighbour_site(site, o, c.ex, c.ey);
    const S* Dr = c.D + (((size_t)site * NOFF + o) * 16 + i) * 16 + 4 * q;
    for (int jj = 0; jj < 4; ++jj) Dv[o][jj] = widen<T>(Dr[jj]);
  }
}
template <typename T>
__device__ __forceinline__ cx<T> coarse_apply_row(const cx<T> (&Dv)[NOFF][4], const int (&nb)[NOFF], int q,
                                                  const cx<T>* __restrict__ xv) {
  cx<T> acc = {0, 0};
  for (int o = 0; o < NOFF; ++o)
    for (int jj = 0; jj < 4; ++jj) acc = acc + Dv[o][jj] * xv[nb[o] * 16 + 4 * q + jj];
  acc = xor_add<1>(acc);
  return xor_add<2>(acc);
}

template <typename T, typename S>
__global__ __launch_bounds__(256) void k_coarse_apply(CoarseT<T, S> c, const cx<T>* __restrict__ x,
                                                      cx<T>* __restrict__ y, const cx<T>* __restrict__ b, int nrhs) {
  using C = cx<T>;
  const int ns = c.ex * c.ey;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int site = blockIdx.x * 4 + wave;
  if (site >= ns) return;
  const int i = lane >> 2, q = lane & 3;
  int nb[NOFF];
  C Dv[NOFF][4];
  coarse_apply_load(c, site, i, q, Dv, nb);
  const size_t n = (size_t)ns * 16;
  for (int r = 0; r < nrhs; ++r) {
    C acc = coarse_apply_row(Dv, nb, q, x + r * n);
    if (q == 0) {
      if (b) acc = b[r * n + site * 16 + i] - acc;
      y[r * n + site * 16 + i] = acc;
    }
  }
}

template <typename T, typename S>
void launch_coarse_apply(const CoarseT<T, S>& c, const cx<T>* x, cx<T>* y, const cx<T>* b, int nrhs, hipStream_t s) {
  int ns = c.ex * c.ey;
  hipLaunchKernelGGL((k_coarse_apply<T, S>), dim3((ns + 3) / 4), dim3(256), 0, s, c, x, y, b, nrhs);
}

// ---------------------------------------------------------------------------
// One colour pass of the coarse Kaczmarz smoother.  The 16 rows d_i of a site
// are projected one after the other (i = 0..15).  With G = A_a A_a^H the
// sequence is exactly alpha = tril(G)^{-1} (b_a - A_a x), x += A_a^H alpha
// (row i sees the updates of rows m < i through G_im), so a work-group
// computes the residual block, applies the precomputed Kinv = tril(G)^{-1}
// and scatters.  128 threads per site: thread (i, q) holds row i, columns
// 2q, 2q+1 of each of the 7 blocks; the column sums of the scatter go
// through LDS.
// ---------------------------------------------------------------------------
// t-th site of coarse colour c (see coarse_ncolours in the host code):
// mode 8: (ax - 3 ay) = c mod 8; mode 16: (ax, ay) = (c mod 4, c / 4) mod 4;
// mode 1: one site per colour.
__device__ __forceinline__ int coarse_colour_site(int c, int mode, int t, int ex) {
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

// One thread's share of a site's projection: row i, columns 2q, 2q+1 of each
// of the NOFF blocks of the block row, the same columns of row i of Kinv, and
// b_i.  The three steps below are the whole projection; every kernel that
// projects coarse sites calls them, so they all give the same bits (products
// with their contraction fixed, sums in a fixed order).
template <typename T>
struct CoarseRow {
  cx<T> Dv[NOFF][2];
  cx<T> k0, k1, bi;
};

template <typename T, typename S>
__device__ __forceinline__ void coarse_row_load(const CoarseT<T, S>& c, int site, int i, int q,
                                                const cx<T>* __restrict__ b, CoarseRow<T>& w) {
  const cx<T>* K = c.Kinv + ((size_t)site * 16 + i) * 16 + 2 * q;
  w.k0 = K[0];
  w.k1 = K[1];
  w.bi = b ? b[site * 16 + i] : cx<T>{0, 0};
#pragma unroll
  for (int o = 0; o < NOFF; ++o) {
    const S* Dr = c.D + (((size_t)site * NOFF + o) * 16 + i) * 16 + 2 * q;
    w.Dv[o][0] = widen<T>(Dr[0]);
    w.Dv[o][1] = widen<T>(Dr[1]);
  }
}

// step 1: rsh[i] = b_i - (A x)_i from the thread's support values xo[o][k]
// (column 2q + k of offset o); 8-lane row sums by DPP moves
template <typename T>
__device__ __forceinline__ void coarse_proj_residual(const CoarseRow<T>& w, const cx<T> (&xo)[NOFF][2], int i, int q,
                                                     cx<T>* rsh) {
  cx<T> acc[NOFF];
#pragma unroll
  for (int o = 0; o < NOFF; ++o) acc[o] = cmul_fixed(w.Dv[o][0], xo[o][0]) + cmul_fixed(w.Dv[o][1], xo[o][1]);
  cx<T> r = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + acc[6]);
  r = xor_add<1>(r);
  r = xor_add<2>(r);
  r = xor_add<4>(r);
  if (q == 0) rsh[i] = w.bi - r;
}

// step 2 (after a barrier): alpha_i = sum_{j <= i} Kinv[i][j] r_j, then
// part[i][col] = conj(D[i][col]) alpha_i for the thread's columns
template <typename T>
__device__ __forceinline__ void coarse_proj_alpha(const CoarseRow<T>& w, const cx<T>* rsh, int i, int q,
                                                  cx<T> (*part)[NOFF * 16 + 1]) {
  cx<T> al = cmul_fixed(w.k0, rsh[2 * q]) + cmul_fixed(w.k1, rsh[2 * q + 1]);
  al = xor_add<1>(al);
  al = xor_add<2>(al);
  al = xor_add<4>(al);
#pragma unroll
  for (int o = 0; o < NOFF; ++o) {
    part[i][o * 16 + 2 * q] = cjmul_fixed(w.Dv[o][0], al);
    part[i][o * 16 + 2 * q + 1] = cjmul_fixed(w.Dv[o][1], al);
  }
}

// step 3 (after a barrier): the update of support column col (offset
// col / 16, component col % 16), the sum over the 16 rows
template <typename T>
__device__ __forceinline__ cx<T> coarse_proj_colsum(const cx<T> (*part)[NOFF * 16 + 1], int col) {
  cx<T> s0 = {0, 0}, s1 = {0, 0};
#pragma unroll
  for (int rr = 0; rr < 16; rr += 2) {
    s0 = s0 + part[rr][col];
    s1 = s1 + part[rr + 1][col];
  }
  return s0 + s1;
}

// (P x_c)[site][d] for level-l site `site` (d = 8 s + j: spin s, row j of
// the site within its 2 x 2 aggregate's 32 rows of spin s), the 8-term sum in
// a fixed order with fixed contractions: the prolongation kernel and the fused
// first post-smoothing launch form it the same way
template <typename T>
__device__ __forceinline__ cx<T> coarse_prolong_entry(int ex, const cx<T>* __restrict__ P, const cx<T>* __restrict__ xc,
                                                      int site, int d) {
  const int cex = ex / 2, s = d >> 3, j = d & 7;
  const int ax = site % ex, ay = site / ex;
  const int A = (ay >> 1) * cex + (ax >> 1), t = 2 * (ay & 1) + (ax & 1);
  const cx<T>* Pr = P + (((size_t)A * 2 + s) * 32 + 8 * t + j) * 8;
  const cx<T>* xcv = xc + A * 16 + 8 * s;
  cx<T> acc = {0, 0};
#pragma unroll
  for (int k = 0; k < 8; ++k) acc = acc + cmul_fixed(Pr[k], xcv[k]);
  return acc;
}

template <typename T, typename S>
__global__ __launch_bounds__(128) void k_kaczmarz_coarse(CoarseT<T, S> c, int colour, int mode, cx<T>* __restrict__ x,
                                                         const cx<T>* __restrict__ b) {
  using C = cx<T>;
  constexpr int dxo[NOFF] = {0, 1, -1, 0, 0, 1, -1};
  constexpr int dyo[NOFF] = {0, 0, 0, 1, -1, 1, -1};
  __shared__ C part[16][NOFF * 16 + 1];
  __shared__ C rsh[16];
  __shared__ C xsh[NOFF * 16];
  const int ns = c.ex * c.ey;
  const int tid = threadIdx.x, i = tid >> 3, q = tid & 7;
  const int site = coarse_colour_site(colour, mode, blockIdx.x, c.ex);
  const int ax = site % c.ex, ay = site / c.ex;
  const size_t n = (size_t)ns * 16;
  C* xv = x + blockIdx.y * n;
  CoarseRow<T> w;
  coarse_row_load(c, site, i, q, b ? b + blockIdx.y * n : nullptr, w);
  int nb[NOFF];
  C xo[NOFF][2];
#pragma unroll
  for (int o = 0; o < NOFF; ++o) {
    nb[o] = cwrap(ay + dyo[o], c.ey) * c.ex + cwrap(ax + dxo[o], c.ex);
    const C* xp = xv + nb[o] * 16 + 2 * q;
    xo[o][0] = xp[0];
    xo[o][1] = xp[1];
  }
  if (i == 0) {
#pragma unroll
    for (int o = 0; o < NOFF; ++o) {
      xsh[o * 16 + 2 * q] = xo[o][0];
      xsh[o * 16 + 2 * q + 1] = xo[o][1];
    }
  }
  coarse_proj_residual(w, xo, i, q, rsh);
  __syncthreads();
  coarse_proj_alpha(w, rsh, i, q, part);
  __syncthreads();
  // thread (i < 14, q) finishes column 2q + (i & 1) of offset i / 2
  if (i < 2 * NOFF) {
    const int o = i >> 1, h = i & 1, col = o * 16 + 2 * q + h;
    // offsets packed as 4-bit fields (+1): (0,0) (+1,0) (-1,0) (0,+1) (0,-1) (+1,+1) (-1,-1)
    const int dx = (int)((0x0211021u >> (4 * o)) & 15u) - 1, dy = (int)((0x0202111u >> (4 * o)) & 15u) - 1;
    const int nbo = cwrap(ay + dy, c.ey) * c.ex + cwrap(ax + dx, c.ex);
    xv[nbo * 16 + 2 * q + h] = xsh[col] + coarse_proj_colsum<T>(part, col);
  }
}

template <typename T, typename S>
void launch_kaczmarz_coarse(const CoarseT<T, S>& c, int colour, int mode, int nsites, cx<T>* x, const cx<T>* b,
                            int nrhs, hipStream_t s) {
  hipLaunchKernelGGL((k_kaczmarz_coarse<T, S>), dim3(nsites, nrhs), dim3(128), 0, s, c, colour, mode, x, b);
}

// ---------------------------------------------------------------------------
// Two colour passes in one launch (8-colouring, colours c and c + 1, c even).
// With the 7-offset stencil, the support of a site s of colour c + 1 meets
// the supports of exactly two sites of colour c, t1 = s + (-1, 0) and
// t2 = s + (2, 1) (the colour differences of the 19 displacements between
// overlapping supports are all distinct, and (ax - 3 ay) mod 8 falls by one
// only for these two).  So the values on the support of s after both passes
// follow from x on the 15 sites of the supports of t1, t2 and s alone: a
// work-group per site s projects t1 and t2 (disjoint supports, together),
// then s, all in LDS, with the three steps of the colour pass (the same
// bits as two colour passes).  Out of place: every work-group reads xin and
// writes xout, the support of s and the site s + (-1, 1), the one site of
// the support of t1 that no colour-(c+1) support holds; these sets tile the
// lattice, so each site is written once (a CPU test checks the claims on
// tori from 8 x 8).  Sites t1 and t2 are projected twice, by the two
// work-groups whose s they neighbour.  256 threads: group 0 projects t1 then
// s, group 1 t2.
// ---------------------------------------------------------------------------
// the 15 sites of a work-group, displacements from s: 0-6 the support of s in
// offset order, 7-9 the rest of the support of t1 ((-2, 0), (-1, 1), (-2, -1)),
// 10-14 that of t2 ((2, 1), (3, 1), (2, 2), (2, 0), (3, 2)); nibble k holds
// dx + 2 and dy + 1 of site k (immediates, not a table in memory: the
// addresses of the first loads and the last stores need no load of their own)
__device__ __forceinline__ int pair_dx(int k) { return (int)((0x544540101322132ull >> (4 * k)) & 15ull) - 2; }
__device__ __forceinline__ int pair_dy(int k) { return (int)((0x313220210202111ull >> (4 * k)) & 15ull) - 1; }
// the support of t1 (t2) in offset order, as local site indices
constexpr int PR_T1 = 2, PR_T2 = 10;
__device__ __forceinline__ int pair_support(int g, int o) {
  constexpr unsigned LT1 = 0x9368702u, LT2 = 0x1EDC5BAu;  // nibble o: local index of offset o
  return (int)(((g ? LT2 : LT1) >> (4 * o)) & 15u);
}

template <typename T, typename S>
__global__ __launch_bounds__(256) void k_kaczmarz_coarse_pair(CoarseT<T, S> c, int colour,
                                                              const cx<T>* __restrict__ xin, cx<T>* __restrict__ xout,
                                                              const cx<T>* __restrict__ b, const cx<T>* __restrict__ P,
                                                              const cx<T>* __restrict__ xc) {
  using C = cx<T>;
  __shared__ C part[2][16][NOFF * 16 + 1];
  __shared__ C rsh[2][16];
  __shared__ C X[15 * 16];
  const int tid = threadIdx.x, g = tid >> 7, i = (tid >> 3) & 15, q = tid & 7;
  const int ex = c.ex, ey = c.ey;
  const int s = coarse_colour_site(colour + 1, 8, (int)xcd_block(blockIdx.x, gridDim.x), ex);
  const int ax = s % ex, ay = s / ex;
  const size_t n = (size_t)ex * ey * 16;
  const C* xr = xin + blockIdx.y * n;
  C* xw = xout + blockIdx.y * n;
  const C* bv = b ? b + blockIdx.y * n : nullptr;
  auto at = [&](int k) { return cwrap(ay + pair_dy(k), ey) * ex + cwrap(ax + pair_dx(k), ex); };
  CoarseRow<T> wt, ws;
  coarse_row_load(c, at(g ? PR_T2 : PR_T1), i, q, bv, wt);
  if (g == 0) coarse_row_load(c, s, i, q, bv, ws);
  if (xc) {  // x + P x_c: the prolongation that precedes the first post-smoothing sweep
    const C* xcv = xc + blockIdx.y * (size_t)(ex / 2) * (ey / 2) * 16;
    for (int e = tid; e < 15 * 16; e += 256) {
      const int site = at(e >> 4);
      X[e] = xr[site * 16 + (e & 15)] + coarse_prolong_entry(ex, P, xcv, site, e & 15);
    }
  } else {
    for (int e = tid; e < 15 * 16; e += 256) X[e] = xr[at(e >> 4) * 16 + (e & 15)];
  }
  __syncthreads();
  // colour c: t1 (group 0) and t2 (group 1)
  {
    C xo[NOFF][2];
#pragma unroll
    for (int o = 0; o < NOFF; ++o) {
      const int e = pair_support(g, o) * 16 + 2 * q;
      xo[o][0] = X[e];
      xo[o][1] = X[e + 1];
    }
    coarse_proj_residual(wt, xo, i, q, rsh[g]);
    __syncthreads();
    coarse_proj_alpha(wt, rsh[g], i, q, part[g]);
    __syncthreads();
    if (i < 2 * NOFF) {
      const int o = i >> 1, h = i & 1, col = o * 16 + 2 * q + h;
      const int e = pair_support(g, o) * 16 + 2 * q + h;
      X[e] = X[e] + coarse_proj_colsum<T>(part[g], col);
    }
    __syncthreads();
  }
  // colour c + 1: s (group 0; group 1 keeps the barriers)
  {
    C xo[NOFF][2];
#pragma unroll
    for (int o = 0; o < NOFF; ++o) {
      xo[o][0] = X[o * 16 + 2 * q];
      xo[o][1] = X[o * 16 + 2 * q + 1];
    }
    if (g == 0) coarse_proj_residual(ws, xo, i, q, rsh[0]);
    __syncthreads();
    if (g == 0) coarse_proj_alpha(ws, rsh[0], i, q, part[0]);
    __syncthreads();
    if (g == 0 && i < 2 * NOFF) {
      const int o = i >> 1, h = i & 1, col = o * 16 + 2 * q + h;
      const int e = o * 16 + 2 * q + h;
      X[e] = X[e] + coarse_proj_colsum<T>(part[0], col);
    }
    __syncthreads();
  }
  // the support of s (local 0-6) and s + (-1, 1) (local 8)
  if (tid < 128) {
    const int k = tid >> 4, loc = k < 7 ? k : 8, e = tid & 15;
    xw[at(loc) * 16 + e] = X[loc * 16 + e];
  }
}

bool coarse_pair_applies(int ex, int ey, int mode) { return mode == 8 && ex >= 8 && ey >= 8 && ex % 8 == 0 && ey % 8 == 0; }

template <typename T, typename S>
void launch_kaczmarz_coarse_pair(const CoarseT<T, S>& c, int colour, int nsites, const cx<T>* xin, cx<T>* xout,
                                 const cx<T>* b, int nrhs, hipStream_t s, const cx<T>* P, const cx<T>* xc) {
  hipLaunchKernelGGL((k_kaczmarz_coarse_pair<T, S>), dim3(nsites, nrhs), dim3(256), 0, s, c, colour, xin, xout, b,
                     P, xc);
}

// ---------------------------------------------------------------------------
// Multi-RHS colour pass on the matrix cores (FP32 arithmetic, operator in its
// storage type S): one wave per site and 16 right-hand sides.  The three
// products of the block form run as real 16x16x4 FP32 MFMA tiles on the real
// and imaginary parts:
//   R = A X       (16 x 112) (112 x 16):  28 K-steps x 4 MFMA
//   alpha = Kinv (B - R)  (16 x 16) (16 x 16): 4 K-steps x 4 MFMA
//   X += A^H alpha  (112 x 16) (16 x 16):  7 tiles x 4 K-steps x 4 MFMA
// MFMA lane layout (v_mfma_f32_16x16x4f32): lane l supplies A[l%16][k0 + l/16]
// and B[k0 + l/16][l%16] and receives C[4(l/16) + e][l%16], e = 0..3.
// The unknowns of the support go through LDS so that the global loads and
// stores run along the site dimension of each right-hand side.
// ---------------------------------------------------------------------------
typedef float mf4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ mf4 mfma4(float a, float b, mf4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename S>
__global__ __launch_bounds__(64) void k_kaczmarz_coarse_mfma(CoarseT<float, S> c, int colour, int mode, int nrhs,
                                                             zf* __restrict__ x, const zf* __restrict__ b) {
  constexpr int NCOL = NOFF * 16, NQ = NCOL * 16 / 64;  // 28 staged unknowns per lane
  __shared__ float Xr[NCOL][17], Xi[NCOL][17];
  __shared__ float Vr[16][17], Vi[16][17];  // right-hand side block, then residual, then alpha
  const int l = threadIdx.x, lm = l & 15, lq = l >> 4;
  const int ns = c.ex * c.ey;
  const size_t n = (size_t)ns * 16;
  const int site = coarse_colour_site(colour, mode, blockIdx.x, c.ex);
  const int r0 = blockIdx.y * 16;
  const int nr = min(16, nrhs - r0);
  const int ax = site % c.ex, ay = site / c.ex;
  int nb[NOFF];
#pragma unroll
  for (int o = 0; o < NOFF; ++o) {
    const int dx = (int)((0x0211021u >> (4 * o)) & 15u) - 1, dy = (int)((0x0202111u >> (4 * o)) & 15u) - 1;
    nb[o] = cwrap(ay + dy, c.ey) * c.ex + cwrap(ax + dx, c.ex);
  }
  // ---- every global load first (independent, all in flight together)
  // unknowns: element e = l + 64 q -> right-hand side e / 112, column e % 112;
  // 64 consecutive elements never straddle more than two offsets
  zf xin[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int e = l + 64 * q, rr = e / NCOL, col = e - rr * NCOL, o = col >> 4;
    int nbo = nb[0];
#pragma unroll
    for (int oo = 1; oo < NOFF; ++oo) nbo = (o == oo) ? nb[oo] : nbo;
    xin[q] = (rr < nr) ? x[(size_t)(r0 + rr) * n + nbo * 16 + (col & 15)] : zf{0, 0};
  }
  const S* Dsite = c.D + (size_t)site * NOFF * 256;
  S ar[NCOL / 4];  // A[lm][4 q + lq]: D[site][q / 4][lm][(4 q + lq) % 16]
#pragma unroll
  for (int q = 0; q < NCOL / 4; ++q) {
    const int k = 4 * q + lq;
    ar[q] = Dsite[(k >> 4) * 256 + lm * 16 + (k & 15)];
  }
  S au[NOFF][4];   // A[4 q + lq][16 o + lm]: D[site][o][4 q + lq][lm]
#pragma unroll
  for (int o = 0; o < NOFF; ++o)
#pragma unroll
    for (int q = 0; q < 4; ++q) au[o][q] = Dsite[o * 256 + (4 * q + lq) * 16 + lm];
  zf kin[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) kin[q] = c.Kinv[(size_t)site * 256 + lm * 16 + 4 * q + lq];
  zf bin[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = l + 64 * q, rr = e >> 4, i = e & 15;
    bin[q] = (b && rr < nr) ? b[(size_t)(r0 + rr) * n + site * 16 + i] : zf{0, 0};
  }
  // ---- stage into LDS
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int e = l + 64 * q, rr = e / NCOL, col = e - rr * NCOL;
    Xr[col][rr] = xin[q].x;
    Xi[col][rr] = xin[q].y;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = l + 64 * q, rr = e >> 4, i = e & 15;
    Vr[i][rr] = bin[q].x;
    Vi[i][rr] = bin[q].y;
  }
  __syncthreads();
  // ---- R = A X
  mf4 cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
#pragma unroll
  for (int q = 0; q < NCOL / 4; ++q) {
    const int k = 4 * q + lq;
    const zf a = widen<float>(ar[q]);
    const float xr = Xr[k][lm], xi = Xi[k][lm];
    cr = mfma4(a.x, xr, cr);
    cr = mfma4(-a.y, xi, cr);
    ci = mfma4(a.x, xi, ci);
    ci = mfma4(a.y, xr, ci);
  }
  float resr[4], resi[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    resr[e] = Vr[4 * lq + e][lm] - cr[e];
    resi[e] = Vi[4 * lq + e][lm] - ci[e];
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    Vr[4 * lq + e][lm] = resr[e];
    Vi[4 * lq + e][lm] = resi[e];
  }
  __syncthreads();
  // ---- alpha = Kinv (B - R)
  mf4 gr = {0, 0, 0, 0}, gi = {0, 0, 0, 0};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int k = 4 * q + lq;
    const zf a = kin[q];
    const float vr = Vr[k][lm], vi = Vi[k][lm];
    gr = mfma4(a.x, vr, gr);
    gr = mfma4(-a.y, vi, gr);
    gi = mfma4(a.x, vi, gi);
    gi = mfma4(a.y, vr, gi);
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    Vr[4 * lq + e][lm] = gr[e];
    Vi[4 * lq + e][lm] = gi[e];
  }
  __syncthreads();
  // ---- X += A^H alpha, tile o: A^H[m][i] = conj(A[i][16 o + m])
#pragma unroll
  for (int o = 0; o < NOFF; ++o) {
    mf4 ur = {0, 0, 0, 0}, ui = {0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = 4 * q + lq;
      const zf a = widen<float>(au[o][q]);
      const float vr = Vr[i][lm], vi = Vi[i][lm];
      // (a.x - i a.y)(vr + i vi) = (a.x vr + a.y vi) + i (a.x vi - a.y vr)
      ur = mfma4(a.x, vr, ur);
      ur = mfma4(a.y, vi, ur);
      ui = mfma4(a.x, vi, ui);
      ui = mfma4(-a.y, vr, ui);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int col = 16 * o + 4 * lq + e;
      Xr[col][lm] += ur[e];
      Xi[col][lm] += ui[e];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int e = l + 64 * q, rr = e / NCOL, col = e - rr * NCOL, o = col >> 4;
    int nbo = nb[0];
#pragma unroll
    for (int oo = 1; oo < NOFF; ++oo) nbo = (o == oo) ? nb[oo] : nbo;
    if (rr < nr) x[(size_t)(r0 + rr) * n + nbo * 16 + (col & 15)] = zf{Xr[col][rr], Xi[col][rr]};
  }
}

// The same colour pass with each (site, 16 right-hand sides) block split over
// the four waves of a 256-thread work-group, so that the matrix-core chain of
// one wave is 76 MFMAs instead of 240: wave w forms the partial residual over
// K-steps 7w .. 7w+6 of the 28, the partials are summed through LDS in wave
// order, every wave forms alpha = Kinv (B - R) from the summed residual, and
// wave w updates the column tiles o = w and w + 4.  The global loads are
// shared by the four waves.
template <typename S>
__global__ __launch_bounds__(256) void k_kaczmarz_coarse_mfma4(CoarseT<float, S> c, int colour, int mode, int nrhs,
                                                               zf* __restrict__ x, const zf* __restrict__ b) {
  constexpr int NCOL = NOFF * 16, NQ = NCOL * 16 / 256;  // 7 staged unknowns per thread
  constexpr int KW = NCOL / 4 / 4;                       // K-steps per wave: 7
  __shared__ float Xr[NCOL][17], Xi[NCOL][17];
  __shared__ float Vr[16][17], Vi[16][17];          // right-hand side block, then the residual
  __shared__ float Pr[4][16][17], Pi[4][16][17];    // partial products of the four waves, then alpha per wave
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, lm = l & 15, lq = l >> 4;
  const int ns = c.ex * c.ey;
  const size_t n = (size_t)ns * 16;
  const int site = coarse_colour_site(colour, mode, blockIdx.x, c.ex);
  const int r0 = blockIdx.y * 16;
  const int nr = min(16, nrhs - r0);
  const int ax = site % c.ex, ay = site / c.ex;
  int nb[NOFF];
#pragma unroll
  for (int o = 0; o < NOFF; ++o) {
    const int dx = (int)((0x0211021u >> (4 * o)) & 15u) - 1, dy = (int)((0x0202111u >> (4 * o)) & 15u) - 1;
    nb[o] = cwrap(ay + dy, c.ey) * c.ex + cwrap(ax + dx, c.ex);
  }
  // ---- every global load first
  zf xin[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int e = tid + 256 * q, rr = e / NCOL, col = e - rr * NCOL, o = col >> 4;
    int nbo = nb[0];
#pragma unroll
    for (int oo = 1; oo < NOFF; ++oo) nbo = (o == oo) ? nb[oo] : nbo;
    xin[q] = (rr < nr) ? x[(size_t)(r0 + rr) * n + nbo * 16 + (col & 15)] : zf{0, 0};
  }
  const S* Dsite = c.D + (size_t)site * NOFF * 256;
  S ar[KW];  // A[lm][4 q + lq] for this wave's K-steps q = KW w + j
#pragma unroll
  for (int j = 0; j < KW; ++j) {
    const int k = 4 * (KW * w + j) + lq;
    ar[j] = Dsite[(k >> 4) * 256 + lm * 16 + (k & 15)];
  }
  S au[2][4];  // A[4 q + lq][16 o + lm] for the tiles o = w, w + 4
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int o = min(w + 4 * t, NOFF - 1);
#pragma unroll
    for (int q = 0; q < 4; ++q) au[t][q] = Dsite[o * 256 + (4 * q + lq) * 16 + lm];
  }
  zf kin[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) kin[q] = c.Kinv[(size_t)site * 256 + lm * 16 + 4 * q + lq];
  zf bin = {0, 0};
  {
    const int rr = tid >> 4, i = tid & 15;
    if (b && rr < nr) bin = b[(size_t)(r0 + rr) * n + site * 16 + i];
  }
  // ---- stage into LDS
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int e = tid + 256 * q, rr = e / NCOL, col = e - rr * NCOL;
    Xr[col][rr] = xin[q].x;
    Xi[col][rr] = xin[q].y;
  }
  {
    const int rr = tid >> 4, i = tid & 15;
    Vr[i][rr] = bin.x;
    Vi[i][rr] = bin.y;
  }
  __syncthreads();
  // ---- partial R = A X over this wave's K-steps
  mf4 cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
#pragma unroll
  for (int j = 0; j < KW; ++j) {
    const int k = 4 * (KW * w + j) + lq;
    const zf a = widen<float>(ar[j]);
    const float xr = Xr[k][lm], xi = Xi[k][lm];
    cr = mfma4(a.x, xr, cr);
    cr = mfma4(-a.y, xi, cr);
    ci = mfma4(a.x, xi, ci);
    ci = mfma4(a.y, xr, ci);
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    Pr[w][4 * lq + e][lm] = cr[e];
    Pi[w][4 * lq + e][lm] = ci[e];
  }
  __syncthreads();
  // ---- residual B - R, the partials summed in wave order (wave 0 writes it)
  float resr[4], resi[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int i = 4 * lq + e;
    const float rr_ = ((Pr[0][i][lm] + Pr[1][i][lm]) + Pr[2][i][lm]) + Pr[3][i][lm];
    const float ri_ = ((Pi[0][i][lm] + Pi[1][i][lm]) + Pi[2][i][lm]) + Pi[3][i][lm];
    resr[e] = Vr[i][lm] - rr_;
    resi[e] = Vi[i][lm] - ri_;
  }
  __syncthreads();
  if (w == 0) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      Vr[4 * lq + e][lm] = resr[e];
      Vi[4 * lq + e][lm] = resi[e];
    }
  }
  __syncthreads();
  // ---- alpha = Kinv (B - R), formed by every wave into its own slot of P
  mf4 gr = {0, 0, 0, 0}, gi = {0, 0, 0, 0};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int k = 4 * q + lq;
    const zf a = kin[q];
    const float vr = Vr[k][lm], vi = Vi[k][lm];
    gr = mfma4(a.x, vr, gr);
    gr = mfma4(-a.y, vi, gr);
    gi = mfma4(a.x, vi, gi);
    gi = mfma4(a.y, vr, gi);
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    Pr[w][4 * lq + e][lm] = gr[e];
    Pi[w][4 * lq + e][lm] = gi[e];
  }
  __syncthreads();
  // ---- X += A^H alpha on the tiles o = w, w + 4 (disjoint columns per wave)
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int o = w + 4 * t;
    if (o < NOFF) {
      mf4 ur = {0, 0, 0, 0}, ui = {0, 0, 0, 0};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = 4 * q + lq;
        const zf a = widen<float>(au[t][q]);
        const float vr = Pr[w][i][lm], vi = Pi[w][i][lm];
        ur = mfma4(a.x, vr, ur);
        ur = mfma4(a.y, vi, ur);
        ui = mfma4(a.x, vi, ui);
        ui = mfma4(-a.y, vr, ui);
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int col = 16 * o + 4 * lq + e;
        Xr[col][lm] += ur[e];
        Xi[col][lm] += ui[e];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int e = tid + 256 * q, rr = e / NCOL, col = e - rr * NCOL, o = col >> 4;
    int nbo = nb[0];
#pragma unroll
    for (int oo = 1; oo < NOFF; ++oo) nbo = (o == oo) ? nb[oo] : nbo;
    if (rr < nr) x[(size_t)(r0 + rr) * n + nbo * 16 + (col & 15)] = zf{Xr[col][rr], Xi[col][rr]};
  }
}

// ---------------------------------------------------------------------------
// y = D x (or y = b - D x) for many right-hand sides on the matrix cores: one
// work-group per site and 16 right-hand sides, the product R = A X of the
// site's 16 x 112 block row with the 112 x 16 support block as real
// 16x16x4 FP32 MFMA tiles split over the four waves by K (7 of the 28
// K-steps each), the partials summed in wave order through LDS.  FP32
// arithmetic, operator in its storage type S, like the smoother above.
// ---------------------------------------------------------------------------
template <typename S>
__global__ __launch_bounds__(256) void k_coarse_apply_mfma4(CoarseT<float, S> c, int nrhs, const zf* __restrict__ x,
                                                            zf* __restrict__ y, const zf* __restrict__ b) {
  constexpr int NCOL = NOFF * 16, NQ = NCOL * 16 / 256;  // 7 staged unknowns per thread
  constexpr int KW = NCOL / 4 / 4;                       // K-steps per wave: 7
  __shared__ float Xr[NCOL][17], Xi[NCOL][17];
  __shared__ float Pr[4][16][17], Pi[4][16][17];  // partial products of the four waves
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, lm = l & 15, lq = l >> 4;
  const int ns = c.ex * c.ey;
  const size_t n = (size_t)ns * 16;
  const int site = blockIdx.x;
  const int r0 = blockIdx.y * 16;
  const int nr = min(16, nrhs - r0);
  const int ax = site % c.ex, ay = site / c.ex;
  int nb[NOFF];
#pragma unroll
  for (int o = 0; o < NOFF; ++o) {
    const int dx = (int)((0x0211021u >> (4 * o)) & 15u) - 1, dy = (int)((0x0202111u >> (4 * o)) & 15u) - 1;
    nb[o] = cwrap(ay + dy, c.ey) * c.ex + cwrap(ax + dx, c.ex);
  }
  // every global load first
  zf xin[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int e = tid + 256 * q, rr = e / NCOL, col = e - rr * NCOL, o = col >> 4;
    int nbo = nb[0];
#pragma unroll
    for (int oo = 1; oo < NOFF; ++oo) nbo = (o == oo) ? nb[oo] : nbo;
    xin[q] = zf{0, 0};
    if (rr < nr) xin[q] = x[(size_t)(r0 + rr) * n + nbo * 16 + (col & 15)];
  }
  const S* Dsite = c.D + (size_t)site * NOFF * 256;
  S ar[KW];  // A[lm][4 q + lq] for this wave's K-steps q = KW w + j
#pragma unroll
  for (int j = 0; j < KW; ++j) {
    const int k = 4 * (KW * w + j) + lq;
    ar[j] = Dsite[(k >> 4) * 256 + lm * 16 + (k & 15)];
  }
  const int orr = tid >> 4, oi = tid & 15;  // the output entry of this thread: right-hand side orr, row oi
  zf bin = {0, 0};
  if (b && orr < nr) bin = b[(size_t)(r0 + orr) * n + site * 16 + oi];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int e = tid + 256 * q, rr = e / NCOL, col = e - rr * NCOL;
    Xr[col][rr] = xin[q].x;
    Xi[col][rr] = xin[q].y;
  }
  __syncthreads();
  mf4 cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
#pragma unroll
  for (int j = 0; j < KW; ++j) {
    const int k = 4 * (KW * w + j) + lq;
    const zf a = widen<float>(ar[j]);
    const float xr = Xr[k][lm], xi = Xi[k][lm];
    cr = mfma4(a.x, xr, cr);
    cr = mfma4(-a.y, xi, cr);
    ci = mfma4(a.x, xi, ci);
    ci = mfma4(a.y, xr, ci);
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    Pr[w][4 * lq + e][lm] = cr[e];
    Pi[w][4 * lq + e][lm] = ci[e];
  }
  __syncthreads();
  if (orr < nr) {
    const float rr_ = ((Pr[0][oi][orr] + Pr[1][oi][orr]) + Pr[2][oi][orr]) + Pr[3][oi][orr];
    const float ri_ = ((Pi[0][oi][orr] + Pi[1][oi][orr]) + Pi[2][oi][orr]) + Pi[3][oi][orr];
    y[(size_t)(r0 + orr) * n + site * 16 + oi] = b ? zf{bin.x - rr_, bin.y - ri_} : zf{rr_, ri_};
  }
}

template <typename S>
void launch_coarse_apply_mfma(const CoarseT<float, S>& c, const zf* x, zf* y, const zf* b, int nrhs, hipStream_t s) {
  hipLaunchKernelGGL((k_coarse_apply_mfma4<S>), dim3(c.ex * c.ey, (nrhs + 15) / 16), dim3(256), 0, s, c, nrhs, x, y,
                     b);
}
template void launch_coarse_apply_mfma<zf>(const CoarseT<float, zf>&, const zf*, zf*, const zf*, int, hipStream_t);
template void launch_coarse_apply_mfma<hcx>(const CoarseT<float, hcx>&, const zf*, zf*, const zf*, int, hipStream_t);
template void launch_coarse_apply_mfma<bcx>(const CoarseT<float, bcx>&, const zf*, zf*, const zf*, int, hipStream_t);

template <typename S>
void launch_kaczmarz_coarse_mfma(const CoarseT<float, S>& c, int colour, int mode, int nsites, zf* x, const zf* b,
                                 int nrhs, hipStream_t s) {
  hipLaunchKernelGGL((k_kaczmarz_coarse_mfma4<S>), dim3(nsites, (nrhs + 15) / 16), dim3(256), 0, s, c, colour, mode,
                     nrhs, x, b);
}
template void launch_kaczmarz_coarse_mfma<zf>(const CoarseT<float, zf>&, int, int, int, zf*, const zf*, int,
                                              hipStream_t);
template void launch_kaczmarz_coarse_mfma<hcx>(const CoarseT<float, hcx>&, int, int, int, zf*, const zf*, int,
                                               hipStream_t);
template void launch_kaczmarz_coarse_mfma<bcx>(const CoarseT<float, bcx>&, int, int, int, zf*, const zf*, int,
                                               hipStream_t);

// ---------------------------------------------------------------------------
// Kinv = tril(G)^{-1}, G = sum_o D[o] D[o]^H per site (G_ii = ||d_i||^2).
// A zero row (G_ii = 0) is skipped by the smoother: its row and column of Kinv
// are zero.
// ---------------------------------------------------------------------------
template <typename T, typename S>
__global__ __launch_bounds__(256) void k_kaczmarz_prep(CoarseT<T, S> c, cx<T>* __restrict__ Kinv) {
  __shared__ zd G[16][16];
  __shared__ zd K[16][16];
  const int site = blockIdx.x;
  const int tid = threadIdx.x, i = tid >> 4, j = tid & 15;
  zd g = {0, 0};
  if (j <= i) {
    for (int o = 0; o < NOFF; ++o) {
      const S* Di = c.D + (((size_t)site * NOFF + o) * 16 + i) * 16;
      const S* Dj = c.D + (((size_t)site * NOFF + o) * 16 + j) * 16;
      for (int m = 0; m < 16; ++m) g = g + cjmul(widen<double>(Dj[m]), widen<double>(Di[m]));
    }
  }
  G[i][j] = g;
  K[i][j] = zd{0, 0};
  __syncthreads();
  if (tid < 16) {
    const int col = tid;
    if (G[col][col].x > 0) {
      K[col][col] = zd{1.0 / G[col][col].x, 0};
      for (int r = col + 1; r < 16; ++r) {
        if (!(G[r][r].x > 0)) continue;
        zd s = {0, 0};
        for (int m = col; m < r; ++m) s = s + G[r][m] * K[m][col];
        K[r][col] = -(cdiv_real(s, G[r][r].x));
      }
    }
  }
  __syncthreads();
  Kinv[((size_t)site * 16 + i) * 16 + j] = cx<T>{(T)K[i][j].x, (T)K[i][j].y};
}

template <typename T, typename S>
void launch_kaczmarz_prep(const CoarseT<T, S>& c, cx<T>* Kinv, hipStream_t s) {
  hipLaunchKernelGGL((k_kaczmarz_prep<T, S>), dim3(c.ex * c.ey), dim3(256), 0, s, c, Kinv);
}

// ---------------------------------------------------------------------------
// 2x2 aggregation: coarse site A = AY*(ex/2) + AX holds the sites
// (2AX + (t&1), 2AY + (t>>1)), local t; P rows 8t + (d mod 8) for spin d/8.
// ---------------------------------------------------------------------------
// (P^H r)[A][d] for coarse dof d = 8 s + k of aggregate A, from rrow(t, e) =
// r[e] of the aggregate's site t; the sum in a fixed order (the restriction
// kernel and the fused residual-restriction kernel form it the same way)
template <typename T, typename F>
__device__ __forceinline__ cx<T> coarse_restrict_entry(const cx<T>* __restrict__ P, int A, int d, F rrow) {
  const int s = d >> 3, k = d & 7;
  const cx<T>* Pa = P + ((size_t)A * 2 + s) * 32 * 8;
  cx<T> acc = {0, 0};
  for (int t = 0; t < 4; ++t)
    for (int j = 0; j < 8; ++j) acc = acc + cjmul(Pa[(8 * t + j) * 8 + k], rrow(t, 8 * s + j));
  return acc;
}

template <typename T>
__global__ void k_restrict_coarse(int ex, int ey, const cx<T>* __restrict__ P, const cx<T>* __restrict__ r,
                                  cx<T>* __restrict__ rc, cx<T>* __restrict__ xz) {
  using C = cx<T>;
  const int cex = ex / 2, cey = ey / 2;
  const int tt = blockIdx.x * blockDim.x + threadIdx.x;
  if (tt >= cex * cey * 16) return;
  const int A = tt >> 4, d = tt & 15;
  const int AX = A % cex, AY = A / cex;
  const size_t n = (size_t)ex * ey * 16, nc = (size_t)cex * cey * 16;
  const C* rv = r + blockIdx.y * n;
  rc[blockIdx.y * nc + tt] = coarse_restrict_entry(P, A, d, [&](int t, int e) {
    return rv[((2 * AY + (t >> 1)) * ex + 2 * AX + (t & 1)) * 16 + e];
  });
  if (xz) xz[blockIdx.y * nc + tt] = C{0, 0};  // the coarser level's zero initial guess
}

// r = b - D x on a coarse level and r_c = P^H r on the next, in one launch: a
// work-group per aggregate A of the next level, wave t forming the residual
// rows of A's site t as k_coarse_apply does (into LDS), then thread d < 16
// the restricted entry d as k_restrict_coarse does: the same bits as the two
// launches, without r in memory.  xz (the next level, may be null) = 0.
template <typename T, typename S>
__global__ __launch_bounds__(256) void k_residual_restrict_coarse(CoarseT<T, S> c, const cx<T>* __restrict__ P,
                                                                  const cx<T>* __restrict__ x,
                                                                  const cx<T>* __restrict__ b,
                                                                  cx<T>* __restrict__ rc, cx<T>* __restrict__ xz) {
  using C = cx<T>;
  __shared__ C rs[4][16];
  const int ex = c.ex, cex = ex / 2, cey = c.ey / 2;
  const int A = blockIdx.x, AX = A % cex, AY = A / cex;
  const int t = threadIdx.x >> 6, lane = threadIdx.x & 63, i = lane >> 2, q = lane & 3;
  const int site = (2 * AY + (t >> 1)) * ex + 2 * AX + (t & 1);
  const size_t n = (size_t)ex * c.ey * 16, nc = (size_t)cex * cey * 16;
  int nb[NOFF];
  C Dv[NOFF][4];
  coarse_apply_load(c, site, i, q, Dv, nb);
  const C acc = coarse_apply_row(Dv, nb, q, x + blockIdx.y * n);
  if (q == 0) rs[t][i] = b[blockIdx.y * n + site * 16 + i] - acc;
  __syncthreads();
  if (threadIdx.x < 16) {
    const int d = threadIdx.x;
    rc[blockIdx.y * nc + (size_t)A * 16 + d] = coarse_restrict_entry(P, A, d, [&](int tt, int e) { return rs[tt][e]; });
    if (xz) xz[blockIdx.y * nc + (size_t)A * 16 + d] = C{0, 0};
  }
}

template <typename T, typename S>
bool launch_residual_restrict_coarse(const CoarseT<T, S>& c, const cx<T>* P, const cx<T>* x, const cx<T>* b,
                                     cx<T>* rc, int nrhs, hipStream_t s, cx<T>* xz) {
  if (!b || nrhs < 1 || c.ex % 2 || c.ey % 2) return false;
  hipLaunchKernelGGL((k_residual_restrict_coarse<T, S>), dim3((c.ex / 2) * (c.ey / 2), nrhs), dim3(256), 0, s, c, P,
                     x, b, rc, xz);
  return true;
}

template <typename T>
void launch_restrict_coarse(int ex, int ey, const cx<T>* P, const cx<T>* r, cx<T>* rc, int nrhs, hipStream_t s,
                            cx<T>* xz) {
  int n = (ex / 2) * (ey / 2) * 16;
  hipLaunchKernelGGL(k_restrict_coarse<T>, dim3((n + 255) / 256, nrhs), dim3(256), 0, s, ex, ey, P, r, rc, xz);
}

template <typename T>
__global__ void k_prolong_coarse(int ex, int ey, const cx<T>* __restrict__ P, const cx<T>* __restrict__ xc,
                                 cx<T>* __restrict__ x) {
  const int tt = blockIdx.x * blockDim.x + threadIdx.x;
  const int ns = ex * ey;
  if (tt >= ns * 16) return;
  const size_t n = (size_t)ns * 16, nc = (size_t)(ex / 2) * (ey / 2) * 16;
  x[blockIdx.y * n + tt] = x[blockIdx.y * n + tt] + coarse_prolong_entry(ex, P, xc + blockIdx.y * nc, tt >> 4, tt & 15);
}

template <typename T>
void launch_prolong_coarse(int ex, int ey, const cx<T>* P, const cx<T>* xc, cx<T>* x, int nrhs, hipStream_t s) {
  int n = ex * ey * 16;
  hipLaunchKernelGGL(k_prolong_coarse<T>, dim3((n + 255) / 256, nrhs), dim3(256), 0, s, ex, ey, P, xc, x);
}

#define BAMG_COARSE_INST(T, S)                                                                          \
  template void launch_coarse_apply<T, S>(const CoarseT<T, S>&, const cx<T>*, cx<T>*, const cx<T>*, int, \
                                          hipStream_t);                                                 \
  template void launch_kaczmarz_coarse<T, S>(const CoarseT<T, S>&, int, int, int, cx<T>*, const cx<T>*, \
                                             int, hipStream_t);                                         \
  template void launch_kaczmarz_prep<T, S>(const CoarseT<T, S>&, cx<T>*, hipStream_t);                  \
  template void launch_kaczmarz_coarse_pair<T, S>(const CoarseT<T, S>&, int, int, const cx<T>*, cx<T>*, \
                                                  const cx<T>*, int, hipStream_t, const cx<T>*, const cx<T>*); \
  template bool launch_residual_restrict_coarse<T, S>(const CoarseT<T, S>&, const cx<T>*, const cx<T>*,  \
                                                      const cx<T>*, cx<T>*, int, hipStream_t, cx<T>*);
BAMG_COARSE_INST(double, zd)
BAMG_COARSE_INST(float, zf)
BAMG_COARSE_INST(float, hcx)
BAMG_COARSE_INST(float, bcx)
#undef BAMG_COARSE_INST
template void launch_restrict_coarse<double>(int, int, const zd*, const zd*, zd*, int, hipStream_t,
                                             zd*);
template void launch_restrict_coarse<float>(int, int, const zf*, const zf*, zf*, int, hipStream_t,
                                             zf*);
template void launch_prolong_coarse<double>(int, int, const zd*, const zd*, zd*, int, hipStream_t);
template void launch_prolong_coarse<float>(int, int, const zf*, const zf*, zf*, int, hipStream_t);

// ---------------------------------------------------------------------------
// Galerkin product of the next level by fine displacement:
// Dc[A][O][(s1,k1),(s2,k2)] = sum_{t, o: agg(a_t + o) = A + O}
//     sum_{j1, j2} conj(P[A][s1][8t+j1][k1]) D[a_t][o][8s1+j1][8s2+j2] P[A+O][s2][8t'+j2][k2]
// ---------------------------------------------------------------------------
__device__ __forceinline__ int fdiv2(int a) { return a >= 0 ? a >> 1 : -((-a + 1) >> 1); }

__global__ __launch_bounds__(256) void k_galerkin_coarse(Coarse c, const zd* __restrict__ P, zd* __restrict__ Dc) {
  const int cex = c.ex / 2, cey = c.ey / 2;
  const int A = blockIdx.x, AX = A % cex, AY = A / cex;
  __shared__ int tO[4][NOFF], tT[4][NOFF], tA[4][NOFF], tS[4];
  const int tid = threadIdx.x;
  if (tid < 4 * NOFF) {
    const int t = tid / NOFF, o = tid - t * NOFF;
    const int ux = 2 * AX + (t & 1), uy = 2 * AY + (t >> 1);
    const int nx = ux + ODX[o], ny = uy + ODY[o];
    const int BX = fdiv2(nx), BY = fdiv2(ny);
    tO[t][o] = coarse_offset_index(BX - AX, BY - AY);
    tT[t][o] = 2 * (ny - 2 * BY) + (nx - 2 * BX);
    tA[t][o] = cwrap(BY, cey) * cex + cwrap(BX, cex);
    if (o == 0) tS[t] = uy * c.ex + ux;
  }
  __syncthreads();
  for (int out = tid; out < NOFF * 256; out += blockDim.x) {
    const int O = out >> 8, rr = (out >> 4) & 15, cc = out & 15;
    const int s1 = rr >> 3, k1 = rr & 7, s2 = cc >> 3, k2 = cc & 7;
    zd acc = {0, 0};
    for (int t = 0; t < 4; ++t)
      for (int o = 0; o < NOFF; ++o) {
        if (tO[t][o] != O) continue;
        const zd* Dblk = c.D + ((size_t)tS[t] * NOFF + o) * 256;
        const zd* Pb = P + ((size_t)tA[t][o] * 2 + s2) * 32 * 8;
        const zd* Pa = P + ((size_t)A * 2 + s1) * 32 * 8;
        for (int j1 = 0; j1 < 8; ++j1) {
          zd part = {0, 0};
          for (int j2 = 0; j2 < 8; ++j2)
            part = part + Dblk[(8 * s1 + j1) * 16 + 8 * s2 + j2] * Pb[(8 * tT[t][o] + j2) * 8 + k2];
          acc = acc + cjmul(Pa[(8 * t + j1) * 8 + k1], part);
        }
      }
    Dc[(((size_t)A * NOFF + O) * 16 + rr) * 16 + cc] = acc;
  }
}

void launch_galerkin_coarse(const Coarse& c, const zd* P, zd* Dc, hipStream_t s) {
  int na = (c.ex / 2) * (c.ey / 2);
  hipLaunchKernelGGL(k_galerkin_coarse, dim3(na), dim3(256), 0, s, c, P, Dc);
}

// ---------------------------------------------------------------------------
// Least-squares fit on a coarse level: 32 rows (4 sites x 8 dofs of spin s)
// per problem, two problems per wave, classical Gram-Schmidt applied twice.
// ---------------------------------------------------------------------------
template <int R>
__device__ __forceinline__ zd seg_sum_c(zd v) {
#pragma unroll
  for (int off = R / 2; off > 0; off >>= 1) v = v + shfl_xor_z(v, off);
  return v;
}

__global__ __launch_bounds__(64) void k_fit_coarse(Coarse c, const zd* __restrict__ V, int k, zd* __restrict__ P) {
  const int cex = c.ex / 2, cey = c.ey / 2;
  const int lane = threadIdx.x, grp = lane >> 5, row = lane & 31;
  const int prob = blockIdx.x * 2 + grp;
  const int nprob = cex * cey * 2;
  const bool act = prob < nprob;
  const int A = act ? prob >> 1 : 0, s = prob & 1;
  const int AX = A % cex, AY = A / cex;
  const int t = row >> 3, j = row & 7;
  const int site = (2 * AY + (t >> 1)) * c.ex + 2 * AX + (t & 1);
  const size_t n = (size_t)c.ex * c.ey * 16;
  zd v[8], qv[8];
  for (int m = 0; m < 8; ++m) v[m] = (act && m < k) ? V[m * n + site * 16 + 8 * s + j] : zd{0, 0};
  for (int m = 0; m < 8; ++m) qv[m] = zd{0, 0};
  for (int jj = 0; jj < k && jj < 8; ++jj) {
    zd w = v[jj];
    for (int pass = 0; pass < 2; ++pass) {
      zd h[8];
      for (int q = 0; q < jj; ++q) h[q] = seg_sum_c<32>(cjmul(qv[q], w));
      for (int q = 0; q < jj; ++q) w = w - qv[q] * h[q];
    }
    const double nrm = sqrt(seg_sum_c<32>(zd{norm2(w), 0.0}).x);
    qv[jj] = nrm > 0 ? cdiv_real(w, nrm) : zd{0, 0};
  }
  if (act)
    for (int m = 0; m < 8; ++m) P[(((size_t)A * 2 + s) * 32 + row) * 8 + m] = qv[m];
}

void launch_fit_coarse(const Coarse& c, const zd* V, int k, zd* P, hipStream_t s) {
  int nprob = (c.ex / 2) * (c.ey / 2) * 2;
  hipLaunchKernelGGL(k_fit_coarse, dim3((nprob + 1) / 2), dim3(64), 0, s, c, V, k, P);
}

// ---------------------------------------------------------------------------
// dense n x n matrix of the block stencil (n = 16 ex ey), aliasing offsets summed
// ---------------------------------------------------------------------------
__global__ void k_densify(Coarse c, zd* __restrict__ A) {
  const int ns = c.ex * c.ey, n = ns * 16;
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= n) return;
  const int site = row >> 4, i = row & 15;
  zd* Ar = A + (size_t)row * n;
  for (int col = 0; col < n; ++col) Ar[col] = zd{0, 0};
  for (int o = 0; o < NOFF; ++o) {
    const int nb = neighbour_site(site, o, c.ex, c.ey);
    const zd* Dr = c.D + (((size_t)site * NOFF + o) * 16 + i) * 16;
    for (int j = 0; j < 16; ++j) Ar[nb * 16 + j] = Ar[nb * 16 + j] + Dr[j];
  }
}

void launch_densify(const Coarse& c, zd* A, hipStream_t s) {
  int n = c.ex * c.ey * 16;
  hipLaunchKernelGGL(k_densify, dim3((n + 63) / 64), dim3(64), 0, s, c, A);
}

}  // namespace bamg
