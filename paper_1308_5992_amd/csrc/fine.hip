// Fine-level kernels: the odd-even reduced Wilson operator Dhat (Sec. 3.2,
// eq. wilsonSchur), the reduction of the right-hand side and the odd-site
// reconstruction, the 16-colour Kaczmarz row projections on Dhat (Sec. 3.1),
// transfer between the fine grid and the first aggregate grid (Sec. 3.3,
// eq. bs), the fine Galerkin product (Sec. 3.5) and the test-vector generator.
//
// Notation: H is the Wilson hopping term of eq. (wilson),
//   (H psi)_z = sum_mu [ P_mu^- U_mu(z) psi_{z+mu} + P_mu^+ conj(U_mu(z-mu)) psi_{z-mu} ],
// P_mu^{+-} = (I +- gamma_mu)/2 with gamma_1 = [[0,1],[1,0]], gamma_2 = [[0,i],[-i,0]]
// (Sec. 2).  Each projector is rank one, so a hop costs one complex product:
//   +x: h = u (a - b) -> (h, -h)        -x: h = u (a + b) -> (h,  h)
//   +y: h = u (a - i b) -> (h, i h)     -y: h = u (a + i b) -> (h, -i h)
// with a factor 1/2 applied once per hop (exact in binary floating point).
#include <algorithm>
#include <vector>

#include "bamg_internal.h"

namespace bamg {

__device__ __forceinline__ int wrapn(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

// half-x index of lattice site (x, y), |displacement| <= N assumed
__device__ __forceinline__ int hidx(int x, int y, int N, int NH) {
  return wrapn(y, N) * NH + (wrapn(x, N) >> 1);
}

// x - k a with one fused multiply-add per component
template <typename T>
__device__ __forceinline__ cx<T> sub_scaled(cx<T> x, T k, cx<T> a) {
  return cx<T>{fma(-k, a.x, x.x), fma(-k, a.y, x.y)};
}

// accumulate the hop in direction d (0:+x 1:-x 2:+y 3:-y) of spinor (a, b) with link u
// (u already conjugated for backward hops) into (o0, o1), without the factor 1/2
template <typename T>
__device__ __forceinline__ void hop_acc(int d, cx<T> u, cx<T> a, cx<T> b, cx<T>& o0, cx<T>& o1) {
  cx<T> h;
  switch (d) {
    case 0: h = cmul_fixed(u, a - b); o0 = o0 + h; o1 = o1 - h; break;
    case 1: h = cmul_fixed(u, a + b); o0 = o0 + h; o1 = o1 + h; break;
    case 2: h = cmul_fixed(u, a - mul_i(b)); o0 = o0 + h; o1 = o1 + mul_i(h); break;
    default: h = cmul_fixed(u, a + mul_i(b)); o0 = o0 + h; o1 = o1 - mul_i(h); break;
  }
}

// ---------------------------------------------------------------------------
// gauge layout: U[mu][y][x] -> Ue/Uo[(y*NH + xh)*2 + mu]
// ---------------------------------------------------------------------------
__global__ void k_gauge_pack(const zd* __restrict__ U, zd* __restrict__ Ue, zd* __restrict__ Uo, int N) {
  int NH = N / 2;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N * NH) return;
  int y = i / NH, xh = i - y * NH, p = y & 1;
  int xe = 2 * xh + p, xo = 2 * xh + 1 - p;
  for (int mu = 0; mu < 2; ++mu) {
    Ue[2 * i + mu] = U[((size_t)mu * N + y) * N + xe];
    Uo[2 * i + mu] = U[((size_t)mu * N + y) * N + xo];
  }
}

void launch_gauge_pack(const zd* U, zd* Ue, zd* Uo, int N, hipStream_t s) {
  int n = N * N / 2;
  hipLaunchKernelGGL(k_gauge_pack, dim3((n + 255) / 256), dim3(256), 0, s, U, Ue, Uo, N);
}

// ---------------------------------------------------------------------------
// bhat = kappa b_e + kappa^2 H_eo b_o   (b in the full-lattice layout)
// ---------------------------------------------------------------------------
__global__ void k_eo_reduce(Fine f, const zd* __restrict__ b, zd* __restrict__ bh) {
  int N = f.N, NH = f.NH;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int r = blockIdx.y;
  if (i >= N * NH) return;
  const zd* bf = b + (size_t)r * 2 * N * N;
  int y = i / NH, xh = i - y * NH;
  int x = 2 * xh + (y & 1);
  const int dx[4] = {1, -1, 0, 0}, dy[4] = {0, 0, 1, -1};
  zd o0 = {0, 0}, o1 = {0, 0};
  for (int d = 0; d < 4; ++d) {
    int xn = wrapn(x + dx[d], N), yn = wrapn(y + dy[d], N);
    size_t q = ((size_t)yn * N + xn) * 2;
    zd u;
    if (d == 0) u = f.Ue[2 * i + 0];
    else if (d == 2) u = f.Ue[2 * i + 1];
    else u = conj(f.Uo[2 * (yn * NH + (xn >> 1)) + (d == 1 ? 0 : 1)]);
    hop_acc(d, u, bf[q], bf[q + 1], o0, o1);
  }
  size_t qe = ((size_t)y * N + x) * 2;
  double k = f.kappa, k2h = 0.5 * f.kappa2;
  zd* out = bh + (size_t)r * N * N;
  out[2 * i] = k * bf[qe] + k2h * o0;
  out[2 * i + 1] = k * bf[qe + 1] + k2h * o1;
}

void launch_eo_reduce(const Fine& f, const zd* b, zd* bh, int nrhs, hipStream_t s) {
  int n = f.N * f.NH;
  hipLaunchKernelGGL(k_eo_reduce, dim3((n + 255) / 256, nrhs), dim3(256), 0, s, f, b, bh);
}

// ---------------------------------------------------------------------------
// x_e copied into the full layout, x_o = kappa b_o + kappa H_oe x_e
// ---------------------------------------------------------------------------
__global__ void k_eo_reconstruct(Fine f, const zd* __restrict__ b, const zd* __restrict__ xe,
                                 zd* __restrict__ x) {
  int N = f.N, NH = f.NH;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int r = blockIdx.y;
  if (i >= N * NH) return;
  const zd* bf = b + (size_t)r * 2 * N * N;
  const zd* xr = xe + (size_t)r * N * N;
  zd* xf = x + (size_t)r * 2 * N * N;
  int y = i / NH, xh = i - y * NH, p = y & 1;
  int lxe = 2 * xh + p, lxo = 2 * xh + 1 - p;
  size_t qe = ((size_t)y * N + lxe) * 2, qo = ((size_t)y * N + lxo) * 2;
  xf[qe] = xr[2 * i];
  xf[qe + 1] = xr[2 * i + 1];
  const int dx[4] = {1, -1, 0, 0}, dy[4] = {0, 0, 1, -1};
  zd o0 = {0, 0}, o1 = {0, 0};
  for (int d = 0; d < 4; ++d) {
    int xn = wrapn(lxo + dx[d], N), yn = wrapn(y + dy[d], N);
    int j = yn * NH + (xn >> 1);
    zd u;
    if (d == 0) u = f.Uo[2 * i + 0];
    else if (d == 2) u = f.Uo[2 * i + 1];
    else u = conj(f.Ue[2 * j + (d == 1 ? 0 : 1)]);
    hop_acc(d, u, xr[2 * j], xr[2 * j + 1], o0, o1);
  }
  double k = f.kappa, kh = 0.5 * f.kappa;
  xf[qo] = k * bf[qo] + kh * o0;
  xf[qo + 1] = k * bf[qo + 1] + kh * o1;
}

void launch_eo_reconstruct(const Fine& f, const zd* b, const zd* xe, zd* x, int nrhs, hipStream_t s) {
  int n = f.N * f.NH;
  hipLaunchKernelGGL(k_eo_reconstruct, dim3((n + 255) / 256, nrhs), dim3(256), 0, s, f, b, xe, x);
}

// ---------------------------------------------------------------------------
// Dhat apply: y = x - kappa^2 H_eo (H_oe x), or y = b - Dhat x.
// One work-group owns a TX x TY tile of even sites (half-x columns x rows).
// Stage 1 computes t = H_oe x on the odd sites of the tile plus a one-site
// halo into LDS; stage 2 applies H_eo from LDS.  x and the links are read
// once from HBM per tile (halo re-reads hit L2).
// ---------------------------------------------------------------------------
// The two stages of k_dhat for one TX x TY tile of even sites at (x0, y0)
// (half-x, y), one site per thread: H_oe x on the odd sites of the tile and
// its one-site halo into LDS (t0, t1: (TY + 2)(TX + 2) entries each), then
// H_eo of that at the thread's site e: (a0, a1) = (H_eo H_oe x)_e without the
// factor kappa^2/4.  The caller finishes y_e = x_e - kappa^2/4 (a0, a1).
template <typename T, int TX, int TY>
__device__ __forceinline__ void dhat_tile_hops(const FineT<T>& f, const cx<T>* __restrict__ xv, cx<T>* t0, cx<T>* t1,
                                               int x0, int y0, cx<T>& a0, cx<T>& a1, int& e) {
  using C = cx<T>;
  constexpr int W = TX + 2, NREG = (TY + 2) * (TX + 2), NT = TX * TY;
  const int N = f.N, NH = f.NH;
  const C* __restrict__ Ue = f.Ue;
  const C* __restrict__ Uo = f.Uo;
  const int tid = threadIdx.x;
  for (int q = tid; q < NREG; q += NT) {
    int cy = q / W, cxh = q - cy * W;
    int yy = wrapn(y0 - 1 + cy, N), xhh = wrapn(x0 - 1 + cxh, NH);
    int lx = 2 * xhh + 1 - (yy & 1);
    int w = yy * NH + xhh;
    int jpx = hidx(lx + 1, yy, N, NH), jmx = hidx(lx - 1, yy, N, NH);
    int jpy = hidx(lx, yy + 1, N, NH), jmy = hidx(lx, yy - 1, N, NH);
    C b0 = {0, 0}, b1 = {0, 0};
    hop_acc(0, Uo[2 * w], xv[2 * jpx], xv[2 * jpx + 1], b0, b1);
    hop_acc(1, conj(Ue[2 * jmx]), xv[2 * jmx], xv[2 * jmx + 1], b0, b1);
    hop_acc(2, Uo[2 * w + 1], xv[2 * jpy], xv[2 * jpy + 1], b0, b1);
    hop_acc(3, conj(Ue[2 * jmy + 1]), xv[2 * jmy], xv[2 * jmy + 1], b0, b1);
    t0[q] = b0;
    t1[q] = b1;
  }
  __syncthreads();
  const int ly = tid / TX, lxh = tid - ly * TX;
  const int yy = y0 + ly, xhh = x0 + lxh, p = yy & 1;
  e = yy * NH + xhh;
  const int qpx = (ly + 1) * W + lxh + 1 + p, qmx = (ly + 1) * W + lxh + p;
  const int qpy = (ly + 2) * W + lxh + 1, qmy = ly * W + lxh + 1;
  const int omx = yy * NH + wrapn(xhh + p - 1, NH), omy = wrapn(yy - 1, N) * NH + xhh;
  a0 = C{0, 0};
  a1 = C{0, 0};
  hop_acc(0, Ue[2 * e], t0[qpx], t1[qpx], a0, a1);
  hop_acc(1, conj(Uo[2 * omx]), t0[qmx], t1[qmx], a0, a1);
  hop_acc(2, Ue[2 * e + 1], t0[qpy], t1[qpy], a0, a1);
  hop_acc(3, conj(Uo[2 * omy + 1]), t0[qmy], t1[qmy], a0, a1);
}

template <typename T, int TX, int TY>
__global__ __launch_bounds__(TX* TY) void k_dhat(FineT<T> f, const cx<T>* __restrict__ x, cx<T>* __restrict__ y,
                                                 const cx<T>* __restrict__ b) {
  using C = cx<T>;
  constexpr int NREG = (TY + 2) * (TX + 2);
  __shared__ C t0[NREG], t1[NREG];
  const size_t n = (size_t)f.N * f.NH * 2;
  const C* __restrict__ xv = x + blockIdx.z * n;
  C a0, a1;
  int e;
  dhat_tile_hops<T, TX, TY>(f, xv, t0, t1, blockIdx.x * TX, blockIdx.y * TY, a0, a1, e);
  const T k2q = (T)(0.25 * f.kappa2);
  C r0 = sub_scaled(xv[2 * e], k2q, a0), r1 = sub_scaled(xv[2 * e + 1], k2q, a1);
  C* yv = y + blockIdx.z * n;
  if (b) {
    const C* bv = b + blockIdx.z * n;
    r0 = bv[2 * e] - r0;
    r1 = bv[2 * e + 1] - r1;
  }
  yv[2 * e] = r0;
  yv[2 * e + 1] = r1;
}

// The residual r = b - Dhat x and its restriction r_c = P^H r in one
// launch, for the tiles of k_dhat with TX = 64, TY = 4: a tile then holds 16
// whole 4 x 4 aggregates (one aggregate row), whose 256 restricted entries
// (2 spins x 8 columns each) are formed from the tile's residual in LDS with
// the arithmetic of k_restrict_fine.  r itself is not stored.  xz (if not
// null) = 0 on the same entries (the coarse level's initial guess).
template <typename T>
__global__ __launch_bounds__(256) void k_residual_restrict_fine(FineT<T> f, const cx<T>* __restrict__ P,
                                                               const cx<T>* __restrict__ x, const cx<T>* __restrict__ b,
                                                               cx<T>* __restrict__ rc, cx<T>* __restrict__ xz) {
  using C = cx<T>;
  constexpr int TX = 64, TY = 4, NREG = (TY + 2) * (TX + 2);
  __shared__ C t0[NREG], t1[NREG];
  __shared__ C rs[TY * TX * 2];  // the tile's residual, [row][half-x][spin]
  const size_t n = (size_t)f.N * f.NH * 2;
  const C* __restrict__ xv = x + blockIdx.z * n;
  const C* __restrict__ bv = b + blockIdx.z * n;
  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
  C a0, a1;
  int e;
  dhat_tile_hops<T, TX, TY>(f, xv, t0, t1, x0, y0, a0, a1, e);
  const T k2q = (T)(0.25 * f.kappa2);
  const C r0 = sub_scaled(xv[2 * e], k2q, a0), r1 = sub_scaled(xv[2 * e + 1], k2q, a1);
  const int tid = threadIdx.x;
  rs[2 * tid] = bv[2 * e] - r0;
  rs[2 * tid + 1] = bv[2 * e + 1] - r1;
  __syncthreads();
  const int cxn = f.NH / 4, cyn = f.N / 4;
  const int al = tid >> 4, d = tid & 15, s = d >> 3, k = d & 7;
  const int a = (y0 / 4) * cxn + x0 / 4 + al;
  const C* Pa = P + ((size_t)a * 2 + s) * 16 * 8;
  C acc = {0, 0};
#pragma unroll
  for (int row = 0; row < 16; ++row) {
    const int ly = row >> 2, lx = row & 3;
    acc = acc + cjmul_fixed(Pa[row * 8 + k], rs[2 * (ly * TX + 4 * al + lx) + s]);
  }
  const size_t nc = (size_t)cxn * cyn * 16;
  rc[blockIdx.z * nc + (size_t)a * 16 + d] = acc;
  if (xz) xz[blockIdx.z * nc + (size_t)a * 16 + d] = C{0, 0};
}

// The same operator for lattices with many tiles: 32 x 16 even sites per
// work-group of 256 threads, right-hand sides looped inside the work-group
// (grid.z splits them into groups), each thread's links and neighbour
// indices loaded once into registers and reused for every right-hand side,
// the odd intermediate double-buffered in LDS (one barrier per right-hand
// side), and each output's own entries loaded before that barrier.  The
// arithmetic is that of k_dhat, term by term.
template <typename T, int TX, int TY>
__global__ __launch_bounds__(256) void k_dhat_tile(FineT<T> f, const cx<T>* __restrict__ x, cx<T>* __restrict__ y,
                                                   const cx<T>* __restrict__ b, int rpg, int nrhs) {
  using C = cx<T>;
  constexpr int NT = 256, W = TX + 2, NREG = (TY + 2) * W;
  constexpr int Q1 = (NREG + NT - 1) / NT, Q2 = TX * TY / NT;
  static_assert(TX * TY % NT == 0, "outputs per thread");
  __shared__ C t0[2][NREG], t1[2][NREG];
  const int N = f.N, NH = f.NH;
  const size_t n = (size_t)N * NH * 2;
  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
  const int tid = threadIdx.x;
  const C* __restrict__ Ue = f.Ue;
  const C* __restrict__ Uo = f.Uo;
  // odd sites of the tile and its one-site halo: neighbours and links
  int j1[Q1][4];
  C l1[Q1][4];
#pragma unroll
  for (int i = 0; i < Q1; ++i) {
    const int q = min(tid + NT * i, NREG - 1);
    const int cy = q / W, cxh = q - cy * W;
    const int yy = wrapn(y0 - 1 + cy, N), xhh = wrapn(x0 - 1 + cxh, NH);
    const int lx = 2 * xhh + 1 - (yy & 1);
    const int w = yy * NH + xhh;
    j1[i][0] = hidx(lx + 1, yy, N, NH);
    j1[i][1] = hidx(lx - 1, yy, N, NH);
    j1[i][2] = hidx(lx, yy + 1, N, NH);
    j1[i][3] = hidx(lx, yy - 1, N, NH);
    l1[i][0] = Uo[2 * w];
    l1[i][1] = conj(Ue[2 * j1[i][1]]);
    l1[i][2] = Uo[2 * w + 1];
    l1[i][3] = conj(Ue[2 * j1[i][3] + 1]);
  }
  // even outputs: LDS slots of the four odd neighbours and links
  int e2[Q2], s2[Q2][4];
  C l2[Q2][4];
#pragma unroll
  for (int k = 0; k < Q2; ++k) {
    const int o = tid + NT * k;
    const int ly = o / TX, lxh = o - ly * TX;
    const int yy = y0 + ly, xhh = x0 + lxh, p = yy & 1;
    const int e = yy * NH + xhh;
    e2[k] = e;
    s2[k][0] = (ly + 1) * W + lxh + 1 + p;
    s2[k][1] = (ly + 1) * W + lxh + p;
    s2[k][2] = (ly + 2) * W + lxh + 1;
    s2[k][3] = ly * W + lxh + 1;
    const int omx = yy * NH + wrapn(xhh + p - 1, NH), omy = wrapn(yy - 1, N) * NH + xhh;
    l2[k][0] = Ue[2 * e];
    l2[k][1] = conj(Uo[2 * omx]);
    l2[k][2] = Ue[2 * e + 1];
    l2[k][3] = conj(Uo[2 * omy + 1]);
  }
  const T k2q = (T)(0.25 * f.kappa2);
  const int rbeg = blockIdx.z * rpg, rend = min(nrhs, rbeg + rpg);
  for (int r = rbeg; r < rend; ++r) {
    const int bb = (r - rbeg) & 1;
    const C* __restrict__ xv = x + (size_t)r * n;
#pragma unroll
    for (int i = 0; i < Q1; ++i) {
      const int q = tid + NT * i;
      if (q < NREG) {
        C a0 = {0, 0}, a1 = {0, 0};
        hop_acc(0, l1[i][0], xv[2 * j1[i][0]], xv[2 * j1[i][0] + 1], a0, a1);
        hop_acc(1, l1[i][1], xv[2 * j1[i][1]], xv[2 * j1[i][1] + 1], a0, a1);
        hop_acc(2, l1[i][2], xv[2 * j1[i][2]], xv[2 * j1[i][2] + 1], a0, a1);
        hop_acc(3, l1[i][3], xv[2 * j1[i][3]], xv[2 * j1[i][3] + 1], a0, a1);
        t0[bb][q] = a0;
        t1[bb][q] = a1;
      }
    }
    C xe[Q2][2], be[Q2][2];
#pragma unroll
    for (int k = 0; k < Q2; ++k) {
      xe[k][0] = xv[2 * e2[k]];
      xe[k][1] = xv[2 * e2[k] + 1];
      if (b) {
        be[k][0] = b[(size_t)r * n + 2 * e2[k]];
        be[k][1] = b[(size_t)r * n + 2 * e2[k] + 1];
      }
    }
    __syncthreads();
    C* __restrict__ yv = y + (size_t)r * n;
#pragma unroll
    for (int k = 0; k < Q2; ++k) {
      C a0 = {0, 0}, a1 = {0, 0};
      hop_acc(0, l2[k][0], t0[bb][s2[k][0]], t1[bb][s2[k][0]], a0, a1);
      hop_acc(1, l2[k][1], t0[bb][s2[k][1]], t1[bb][s2[k][1]], a0, a1);
      hop_acc(2, l2[k][2], t0[bb][s2[k][2]], t1[bb][s2[k][2]], a0, a1);
      hop_acc(3, l2[k][3], t0[bb][s2[k][3]], t1[bb][s2[k][3]], a0, a1);
      C r0 = sub_scaled(xe[k][0], k2q, a0), r1 = sub_scaled(xe[k][1], k2q, a1);
      if (b) {
        r0 = be[k][0] - r0;
        r1 = be[k][1] - r1;
      }
      yv[2 * e2[k]] = r0;
      yv[2 * e2[k] + 1] = r1;
    }
  }
}

// The same operator streamed: one wave per (strip, segment, right-hand
// side).  A strip is 64 consecutive half-x columns, lane l on column
// 62 s - 1 + l; lanes 1..62 write, lanes 0 and 63 carry the halo columns
// whose odd intermediate the edge outputs need.  The wave marches down the H
// rows of its segment: per row it loads one coalesced row segment of x and
// of both link arrays, forms the odd intermediate of that row (the +-x even
// neighbours from the adjacent lanes, the +-y ones from its own ring of
// three x rows) and then the output of the row above it (the +-x odd
// neighbours again from the adjacent lanes, the +-y ones from its ring of
// three intermediate rows).  No LDS, no barriers; each entry is read once
// per segment, apart from 2 rows of x and the 2 halo columns.  The
// arithmetic is that of k_dhat, term by term.
constexpr int STRIP = 62;

template <typename T>
__device__ __forceinline__ cx<T> shfl_up1(cx<T> v) {
  return cx<T>{__shfl_up(v.x, 1, 64), __shfl_up(v.y, 1, 64)};
}
template <typename T>
__device__ __forceinline__ cx<T> shfl_down1(cx<T> v) {
  return cx<T>{__shfl_down(v.x, 1, 64), __shfl_down(v.y, 1, 64)};
}

template <typename T>
struct DhatRow {
  cx<T> x0, x1, e0, e1, o0, o1;  // x (both spins), Ue and Uo (both directions) of one row at this lane's column
};

// NTS: non-temporal stores of y (outputs far larger than the caches: they are
// not re-read by this launch, and allocating them in L2 / the Infinity Cache
// only evicts the x and link rows that the neighbouring segments still read)
template <typename T, int PF, bool NTS>
__global__ __launch_bounds__(256) void k_dhat_strip(FineT<T> f, const cx<T>* __restrict__ x, cx<T>* __restrict__ y,
                                                    const cx<T>* __restrict__ b, int nstrips, int H, int nseg,
                                                    int nrhs) {
  using C = cx<T>;
  using Row = DhatRow<T>;
  constexpr int U = 3 + PF;  // row slots: rows ty-1, ty, ty+1 and PF rows in flight
  const int lane = threadIdx.x & 63;
  // consecutive items: right-hand sides, then strips across the lattice, then
  // segments; each XCD takes one contiguous range of them (a band of whole
  // rows), so a segment's halo rows are rows that the segments above and
  // below it load through the same L2
  const long item = (long)xcd_block(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
  if (item >= (long)nstrips * nseg * nrhs) return;  // whole waves leave together
  const int r = (int)(item % nrhs);
  const long sg = item / nrhs;
  const int strip = (int)(sg % nstrips), seg = (int)(sg / nstrips);
  const int N = f.N, NH = f.NH;
  const size_t n = (size_t)N * NH * 2;
  const int cl = strip * STRIP - 1 + lane;  // column of this lane before wrapping; NH >= 64
  const int c = cl < 0 ? cl + NH : (cl >= NH ? cl - NH : cl);
  const bool writes = lane >= 1 && lane <= STRIP && cl < NH;
  const int y0 = seg * H;
  const C* __restrict__ xv = x + (size_t)r * n;
  const C* __restrict__ bv = b ? b + (size_t)r * n : nullptr;
  C* __restrict__ yv = y + (size_t)r * n;
  const C* __restrict__ Ue = f.Ue;
  const C* __restrict__ Uo = f.Uo;
  const T k2q = (T)(0.25 * f.kappa2);
  auto at = [&](int yy) { return 2 * ((size_t)wrapn(yy, N) * NH + c); };
  auto load = [&](int yy) {
    const size_t i = at(yy);
    return Row{xv[i], xv[i + 1], Ue[i], Ue[i + 1], Uo[i], Uo[i + 1]};
  };
  // slot k holds row y0 - 2 + m for the latest m = k (mod U) loaded; step g
  // (t row ty = y0 - 1 + g) reads rows m = g, g+1, g+2 and loads m = g+2+PF
  // into the slot of m = g-1, which step g-1 was the last to read.  The march
  // is unrolled by U so that every slot is a fixed register set, and a row is
  // first read PF steps after its load was issued.
  Row S[U];
#pragma unroll
  for (int k = 0; k < U - 1; ++k) S[k] = load(y0 - 2 + k);
  C uomm1 = {0, 0}, tmm0 = {0, 0}, tmm1 = {0, 0}, tm0 = {0, 0}, tm1 = {0, 0};
  C bn0 = {0, 0}, bn1 = {0, 0};
  const int steps = H + 2, last = y0 + H + 1;  // t rows y0-1 .. y0+H; rows used up to y0+H+1
  for (int g0 = 0; g0 < steps; g0 += U) {
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int g = g0 + j;
      if (g < steps) {
        const int ty = y0 - 1 + g;
        Row& rm = S[j % U];
        Row& r0 = S[(j + 1) % U];
        Row& rp = S[(j + 2) % U];
        if (ty + 1 + PF <= last) S[(j + U - 1) % U] = load(ty + 1 + PF);  // into the slot of row ty-2
        const int p = ty & 1;  // N is even, so the parity survives the wrap
        // odd intermediate of row ty
        C xpx0, xpx1, xmx0, xmx1, uex;
        if (p) {
          xpx0 = r0.x0; xpx1 = r0.x1;
          xmx0 = shfl_up1(r0.x0); xmx1 = shfl_up1(r0.x1);
          uex = shfl_up1(r0.e0);
        } else {
          xpx0 = shfl_down1(r0.x0); xpx1 = shfl_down1(r0.x1);
          xmx0 = r0.x0; xmx1 = r0.x1;
          uex = r0.e0;
        }
        C t0 = {0, 0}, t1 = {0, 0};
        hop_acc(0, r0.o0, xpx0, xpx1, t0, t1);
        hop_acc(1, conj(uex), xmx0, xmx1, t0, t1);
        hop_acc(2, r0.o1, rp.x0, rp.x1, t0, t1);
        hop_acc(3, conj(rm.e1), rm.x0, rm.x1, t0, t1);
        // output of row ty - 1 (parity 1 - p)
        if (ty >= y0 + 1) {
          C tpx0, tpx1, tmx0, tmx1, uox;
          if (p) {
            tpx0 = tm0; tpx1 = tm1;
            tmx0 = shfl_up1(tm0); tmx1 = shfl_up1(tm1);
            uox = shfl_up1(rm.o0);
          } else {
            tpx0 = shfl_down1(tm0); tpx1 = shfl_down1(tm1);
            tmx0 = tm0; tmx1 = tm1;
            uox = rm.o0;
          }
          C a0 = {0, 0}, a1 = {0, 0};
          hop_acc(0, rm.e0, tpx0, tpx1, a0, a1);
          hop_acc(1, conj(uox), tmx0, tmx1, a0, a1);
          hop_acc(2, rm.e1, t0, t1, a0, a1);
          hop_acc(3, conj(uomm1), tmm0, tmm1, a0, a1);
          C r0v = sub_scaled(rm.x0, k2q, a0), r1v = sub_scaled(rm.x1, k2q, a1);
          if (bv) {
            r0v = bn0 - r0v;
            r1v = bn1 - r1v;
          }
          if (writes) {
            const size_t i = at(ty - 1);
            if constexpr (NTS) {
              __builtin_nontemporal_store(r0v.x, &yv[i].x);
              __builtin_nontemporal_store(r0v.y, &yv[i].y);
              __builtin_nontemporal_store(r1v.x, &yv[i + 1].x);
              __builtin_nontemporal_store(r1v.y, &yv[i + 1].y);
            } else {
              yv[i] = r0v;
              yv[i + 1] = r1v;
            }
          }
        }
        if (bv && ty < y0 + H) {  // right-hand side of the next output row, ty
          const size_t i = at(ty);
          bn0 = bv[i];
          bn1 = bv[i + 1];
        }
        tmm0 = tm0; tmm1 = tm1; tm0 = t0; tm1 = t1;
        uomm1 = rm.o1;
      }
    }
  }
}

// the streamed strips (0), the 32 x 16 tiles with the right-hand-side loop
// (1) or the small tiles (2) for launch_dhat
static int dhat_form(int N, int NH, int nrhs, size_t tsize) {
  if (NH >= 64) {
    const int S = (NH + STRIP - 1) / STRIP;
    const int H = tsize == 8 ? 16 : 64;
    const long items = (N % H == 0) ? (long)S * (N / H) * nrhs : 0;
    if (items >= 2048 && (tsize == 8 || nrhs <= 4)) return 0;
  }
  if (NH % 32 == 0 && N % 16 == 0 && (NH / 32) * (N / 16) >= 256) return 1;
  return 2;
}

template <typename T>
void launch_dhat(const FineT<T>& f, const cx<T>* x, cx<T>* y, const cx<T>* b, int nrhs, hipStream_t s) {
  const int N = f.N, NH = f.NH;
  // Kernel choice by measured speed (all three give the same bits): FP64
  // streams 16-row strip segments when they make >= 2048 waves (32- and
  // 64-row segments were slower: fewer waves in flight); FP32 streams
  // 64-row segments for up to 4 right-hand sides when they make >= 2048
  // waves, and otherwise uses the 32 x 16 tiles, whose right-hand-side loop
  // keeps the links in registers.  Outputs of 128 MiB and more are stored
  // non-temporally (4096^2: 4.67 -> 4.84 TB/s in compulsory bytes, 512^2 x 64:
  // 3.1 -> 3.5; at 2048^2, 64 MiB, the cached stores are faster).
  if (NH >= 64) {
    const int S = (NH + STRIP - 1) / STRIP;
    const int H = sizeof(T) == 8 ? 16 : 64;
    const long items = (N % H == 0) ? (long)S * (N / H) * nrhs : 0;
    if (items >= 2048 && (sizeof(T) == 8 || nrhs <= 4)) {
      const bool nts = (size_t)N * N * nrhs * sizeof(cx<T>) >= ((size_t)128 << 20);
      if (nts)
        hipLaunchKernelGGL((k_dhat_strip<T, 1, true>), dim3((unsigned)((items + 3) / 4)), dim3(256), 0, s, f, x, y, b,
                           S, H, N / H, nrhs);
      else
        hipLaunchKernelGGL((k_dhat_strip<T, 1, false>), dim3((unsigned)((items + 3) / 4)), dim3(256), 0, s, f, x, y,
                           b, S, H, N / H, nrhs);
      return;
    }
  }
  constexpr int TTX = 32, TTY = 16;
  if (NH % TTX == 0 && N % TTY == 0) {
    const int tiles = (NH / TTX) * (N / TTY);
    if (tiles >= 256) {  // enough work-groups without splitting the lattice finer
      const int groups = std::max(1, std::min(nrhs, (1024 + tiles - 1) / tiles));
      const int rpg = (nrhs + groups - 1) / groups;
      const dim3 g(NH / TTX, N / TTY, (nrhs + rpg - 1) / rpg);
      hipLaunchKernelGGL((k_dhat_tile<T, TTX, TTY>), g, dim3(256), 0, s, f, x, y, b, rpg, nrhs);
      return;
    }
  }
  dim3 g;
#define DHAT_CASE(TX)                                                                     \
  if (NH % TX == 0) {                                                                     \
    g = dim3(NH / TX, N / 4, nrhs);                                                       \
    hipLaunchKernelGGL((k_dhat<T, TX, 4>), g, dim3(TX * 4), 0, s, f, x, y, b);              \
    return;                                                                               \
  }
  DHAT_CASE(64) DHAT_CASE(32) DHAT_CASE(16) DHAT_CASE(8) DHAT_CASE(4)
#undef DHAT_CASE
}
template void launch_dhat<double>(const FineT<double>&, const zd*, zd*, const zd*, int, hipStream_t);
template void launch_dhat<float>(const FineT<float>&, const zf*, zf*, const zf*, int, hipStream_t);

template <typename T>
bool launch_residual_restrict_fine(const FineT<T>& f, const cx<T>* P, const cx<T>* x, const cx<T>* b, cx<T>* rc,
                                   int nrhs, hipStream_t s, cx<T>* xz) {
  // only where launch_dhat takes the small tiles (the other forms are faster
  // on larger lattices)
  if (f.NH % 64 != 0 || f.N % 4 != 0 || !b || nrhs < 1 || dhat_form(f.N, f.NH, nrhs, sizeof(T)) != 2) return false;
  hipLaunchKernelGGL(k_residual_restrict_fine<T>, dim3(f.NH / 64, f.N / 4, nrhs), dim3(256), 0, s, f, P, x, b, rc, xz);
  return true;
}
template bool launch_residual_restrict_fine<double>(const FineT<double>&, const zd*, const zd*, const zd*, zd*, int,
                                                    hipStream_t, zd*);
template bool launch_residual_restrict_fine<float>(const FineT<float>&, const zf*, const zf*, const zf*, zf*, int,
                                                   hipStream_t, zf*);

// ---------------------------------------------------------------------------
// Rows of Dhat at even site (xh, y): e[n][s][t] = Dhat[(i,s), (j_n,t)] for the
// nine even sites j_n at lattice displacement (SDX[n], SDY[n]).  Built from
// the two-hop paths i -> w -> j; back-tracking paths vanish exactly
// (P^- P^+ = 0) and are skipped, so the diagonal block is I.
// ---------------------------------------------------------------------------
__constant__ int SDX[9] = {0, 2, -2, 0, 0, 1, 1, -1, -1};
__constant__ int SDY[9] = {0, 0, 0, 2, -2, 1, -1, 1, -1};
// slot of the path (d1, d2), -1 for back-tracking
__constant__ int SLOT[4][4] = {{1, -1, 5, 6}, {-1, 2, 7, 8}, {5, 7, 3, -1}, {6, 8, -1, 4}};

// 2x2 projector (times 2) of the hop in direction d: Pi_d = 2 P^{-+}
__device__ __forceinline__ void proj2(int d, zd P[2][2]) {
  const zd one = {1, 0}, mone = {-1, 0}, I = {0, 1}, mI = {0, -1};
  switch (d) {
    case 0: P[0][0] = one; P[0][1] = mone; P[1][0] = mone; P[1][1] = one; break;  // I - g1
    case 1: P[0][0] = one; P[0][1] = one; P[1][0] = one; P[1][1] = one; break;    // I + g1
    case 2: P[0][0] = one; P[0][1] = mI; P[1][0] = I; P[1][1] = one; break;       // I - g2
    default: P[0][0] = one; P[0][1] = I; P[1][0] = mI; P[1][1] = one; break;      // I + g2
  }
}

__device__ void dhat_rows(const Fine& f, int xh, int y, zd e[9][2][2], int jn[9]) {
  const int N = f.N, NH = f.NH;
  const int x = 2 * xh + (y & 1);
  const int i = y * NH + xh;
  const int dxs[4] = {1, -1, 0, 0}, dys[4] = {0, 0, 1, -1};
  for (int n = 0; n < 9; ++n) {
    jn[n] = hidx(x + SDX[n], y + SDY[n], N, NH);
    for (int s = 0; s < 2; ++s)
      for (int t = 0; t < 2; ++t) e[n][s][t] = zd{0, 0};
  }
  for (int d1 = 0; d1 < 4; ++d1) {
    const int wx = x + dxs[d1], wy = y + dys[d1];
    const int w = hidx(wx, wy, N, NH);
    zd l1;
    if (d1 == 0) l1 = f.Ue[2 * i];
    else if (d1 == 2) l1 = f.Ue[2 * i + 1];
    else l1 = conj(f.Uo[2 * w + (d1 == 1 ? 0 : 1)]);
    zd P1[2][2];
    proj2(d1, P1);
    for (int d2 = 0; d2 < 4; ++d2) {
      const int sl = SLOT[d1][d2];
      if (sl < 0) continue;
      zd l2;
      if (d2 == 0) l2 = f.Uo[2 * w];
      else if (d2 == 2) l2 = f.Uo[2 * w + 1];
      else l2 = conj(f.Ue[2 * jn[sl] + (d2 == 1 ? 0 : 1)]);
      zd P2[2][2];
      proj2(d2, P2);
      const zd u = l1 * l2;
      for (int s = 0; s < 2; ++s)
        for (int t = 0; t < 2; ++t) {
          zd pp = P1[s][0] * P2[0][t] + P1[s][1] * P2[1][t];
          e[sl][s][t] = e[sl][s][t] + pp * u;
        }
    }
  }
  // Dhat = I - kappa^2 H_eo H_oe, each hop carrying 1/2
  const double k2q = 0.25 * f.kappa2;
  for (int n = 0; n < 9; ++n)
    for (int s = 0; s < 2; ++s)
      for (int t = 0; t < 2; ++t) e[n][s][t] = -(k2q * e[n][s][t]);
  e[0][0][0] = e[0][0][0] + zd{1, 0};
  e[0][1][1] = e[0][1][1] + zd{1, 0};
}

// ---------------------------------------------------------------------------
// One colour pass of the fine Kaczmarz smoother: every site of the colour
// projects its spin-0 row, then its spin-1 row:
//   alpha = (b_r - d_r . x) / ||d_r||^2,  x_j += alpha conj(d_rj).
// Sites of one colour touch disjoint sets of unknowns.
//
// A group of 16 lanes owns one site; lane n < 9 owns stencil slot n (the even
// site at displacement (SLOT_DX2, SLOT_DY2 field n) - 2): it builds the 2x2 block of Dhat
// coupling the site to slot n from the one or two two-hop paths that reach
// it, and holds the two unknowns of that slot.  With G10 = d_1 d_0^H the two
// sequential projections are
//   alpha_0 = (b_0 - d_0 x) / nu_0,
//   alpha_1 = (b_1 - d_1 x - G10 alpha_0) / nu_1,
// so one group reduction of (d_0 x, d_1 x, nu_0, nu_1, G10) suffices.
// ---------------------------------------------------------------------------
// The coefficients of a site's two sequential row projections:
// alpha_0 = e_0 / nu_0 and alpha_1 = (e_1 - G10 alpha_0) / nu_1 (e_i the row
// residuals).  In FP32 as products with 1 / nu: the reciprocals depend only on
// the stored norms, so they leave the residual's dependency chain (the FP32
// sweep at 256^2: 17.7 -> 16.3 us); in FP64 as quotients (the reciprocals
// measured slower there).  Every form of the fine sweep forms them here and
// so agrees bitwise; a zero norm gives a zero coefficient.
template <typename T>
__device__ __forceinline__ void kz_coefs(cx<T> nu, cx<T> g10, cx<T> e0, cx<T> e1, cx<T>& a0, cx<T>& a1) {
  if constexpr (sizeof(T) == 4) {
    const T i0 = nu.x > 0 ? T(1) / nu.x : T(0), i1 = nu.y > 0 ? T(1) / nu.y : T(0);
    a0 = nu.x > 0 ? cx<T>{e0.x * i0, e0.y * i0} : cx<T>{0, 0};
    const cx<T> f1 = e1 - cmul_fixed(g10, a0);
    a1 = nu.y > 0 ? cx<T>{f1.x * i1, f1.y * i1} : cx<T>{0, 0};
  } else {
    a0 = nu.x > 0 ? cdiv_real(e0, nu.x) : cx<T>{0, 0};
    a1 = nu.y > 0 ? cdiv_real(e1 - cmul_fixed(g10, a0), nu.y) : cx<T>{0, 0};
  }
}

// Per-slot tables packed in 4-bit fields so that a lane-dependent lookup is
// pure register arithmetic: displacement + 2 of slot n, and d + 1 of the
// first / second hop of the (up to two) two-hop paths reaching slot n.
constexpr uint64_t SLOT_DX2 = 0x113322042ull, SLOT_DY2 = 0x131304222ull;
constexpr uint64_t PATH_A1 = 0x221143210ull, PATH_B1 = 0x434300000ull;  // path 0 / 1, first hop
constexpr uint64_t PATH_A2 = 0x434343210ull, PATH_B2 = 0x221100000ull;  // path 0 / 1, second hop
__device__ __forceinline__ int nib(uint64_t c, int n) { return (int)((c >> (4 * n)) & 15ull); }

// Sum over a 16-lane group (a DPP row): the xor butterfly over lane offsets
// 8, 4, 2, 1, each lane adding its partner's value to its own.  The partners
// are read with DPP moves: xor 8 as a row rotation by 8; xor 4 as a row
// rotation by 4, which reads the same value because after the first step
// lanes i and i ^ 8 hold equal sums; xor 2 and xor 1 as quad permutations.
// Every lane adds the same pairs in the same order as the xor butterfly, so
// the sums (and every kernel that reproduces that order) keep their bits.

template <typename T>
__device__ __forceinline__ cx<T> grp16_sum(cx<T> v) {
  v.x += dpp_mov<DPP_ROW_ROR8>(v.x);
  v.y += dpp_mov<DPP_ROW_ROR8>(v.y);
  v.x += dpp_mov<DPP_ROW_ROR4>(v.x);
  v.y += dpp_mov<DPP_ROW_ROR4>(v.y);
  v.x += dpp_mov<DPP_QUAD_XOR2>(v.x);
  v.y += dpp_mov<DPP_QUAD_XOR2>(v.y);
  v.x += dpp_mov<DPP_QUAD_XOR1>(v.x);
  v.y += dpp_mov<DPP_QUAD_XOR1>(v.y);
  return v;
}

// 2x2 block of Dhat between even site (x, y) (half-x index i) and its slot n
// (half-x index jn): -kappa^2/4 sum over paths of Pi_{d1} Pi_{d2} u1 u2, plus I
// on slot 0.  Pi_d = 2 P = [[1, a], [conj(a), 1]] with a = -1, 1, -i, i for
// d = +x, -x, +y, -y, so Pi_1 Pi_2 = [[1 + a1 conj(a2), a1 + a2],
// [conj(a1 + a2), 1 + conj(a1) a2]]; links are selected without branches.
template <typename T>
__device__ __forceinline__ cx<T> hop_phase(int d) {
  const T sg = (d & 1) ? T(1) : T(-1);
  return (d < 2) ? cx<T>{sg, T(0)} : cx<T>{T(0), sg};
}

template <typename T>
__device__ __forceinline__ void dhat_slot_block(const FineT<T>& f, int x, int y, int i, int n, int jn, cx<T> B[2][2]) {
  using C = cx<T>;
  const int N = f.N, NH = f.NH;
  C b00 = {0, 0}, b01 = {0, 0}, b10 = {0, 0}, b11 = {0, 0};
#pragma unroll
  for (int pth = 0; pth < 2; ++pth) {
    const int d1 = nib(pth ? PATH_B1 : PATH_A1, n) - 1, d2 = nib(pth ? PATH_B2 : PATH_A2, n) - 1;
    if (d1 >= 0) {
      const int dx1 = d1 == 0 ? 1 : (d1 == 1 ? -1 : 0), dy1 = d1 == 2 ? 1 : (d1 == 3 ? -1 : 0);
      const int w = hidx(x + dx1, y + dy1, N, NH);
      const bool bk1 = d1 & 1, bk2 = d2 & 1;
      // first hop: forward link at i (even) or conj of the link at w (odd);
      // second hop: forward link at w (odd) or conj of the link at jn (even)
      const C* p1 = bk1 ? f.Uo + 2 * w + (d1 >> 1) : f.Ue + 2 * i + (d1 >> 1);
      const C* p2 = bk2 ? f.Ue + 2 * jn + (d2 >> 1) : f.Uo + 2 * w + (d2 >> 1);
      C l1 = *p1, l2 = *p2;
      l1.y = bk1 ? -l1.y : l1.y;
      l2.y = bk2 ? -l2.y : l2.y;
      // the one inexact product of a path, with its contraction fixed; the
      // phase factors below are 0, +-1, +-2, +-i, so their products are exact
      // and the result does not depend on how the compiler fuses them (the
      // blocks are formed both at setup and inside the pipelined sweep, with
      // the same bits)
      const C u = cmul_fixed(l1, l2);
      const C a1 = hop_phase<T>(d1), a2 = hop_phase<T>(d2);
      const C s12 = a1 + a2;
      b00 = b00 + (C{1, 0} + a1 * conj(a2)) * u;
      b01 = b01 + s12 * u;
      b10 = b10 + conj(s12) * u;
      b11 = b11 + (C{1, 0} + conj(a1) * a2) * u;
    }
  }
  const T k2q = (T)(0.25 * f.kappa2);
  const T one = (n == 0) ? T(1) : T(0);
  B[0][0] = C{fma(-k2q, b00.x, one), -(k2q * b00.y)};
  B[0][1] = -(k2q * b01);
  B[1][0] = -(k2q * b10);
  B[1][1] = C{fma(-k2q, b11.x, one), -(k2q * b11.y)};
}

// The slot blocks of every even site, stored once at setup (and after the
// links change): Bst[site][slot][4] = (B00, B01, B10, B11).  The smoother
// reads them instead of rebuilding them from the links in every pass.
template <typename T>
__global__ void k_slot_blocks(FineT<T> f, cx<T>* __restrict__ Bst) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= f.N * f.NH * 16) return;
  const int i = t >> 4, slot = t & 15;
  if (slot >= 9) return;
  const int y = i / f.NH, xh = i - y * f.NH, px = 2 * xh + (y & 1);
  const int jn = hidx(px + nib(SLOT_DX2, slot) - 2, y + nib(SLOT_DY2, slot) - 2, f.N, f.NH);
  cx<T> B[2][2];
  dhat_slot_block(f, px, y, i, slot, jn, B);
  cx<T>* o = Bst + ((size_t)i * 9 + slot) * 4;
  o[0] = B[0][0];
  o[1] = B[0][1];
  o[2] = B[1][0];
  o[3] = B[1][1];
}

template <typename T>
void launch_slot_blocks(const FineT<T>& f, cx<T>* Bst, hipStream_t s) {
  const int n = f.N * f.NH * 16;
  hipLaunchKernelGGL(k_slot_blocks<T>, dim3((n + 255) / 256), dim3(256), 0, s, f, Bst);
}
template void launch_slot_blocks<double>(const FineT<double>&, zd*, hipStream_t);
template void launch_slot_blocks<float>(const FineT<float>&, zf*, hipStream_t);

// t-th even site of fine colour c = 4a + b (a = (x+y)/2 mod 4, b = (x-y)/2 mod 4):
// rows y = a - b (mod 4), and in such a row x = 2a - y (mod 8); N^2/32 sites.
__device__ __forceinline__ void fine_colour_site(int c, int t, int N, int& x, int& y) {
  const int a = c >> 2, b = c & 3, per = N >> 3;
  const int r = t / per, k = t - r * per;
  y = 4 * r + ((a - b) & 3);
  x = 8 * k + ((2 * a - y) & 7);
}

template <typename T>
__device__ __forceinline__ T norm2_fixed(cx<T> a) {
  return fma(a.x, a.x, a.y * a.y);
}

// ((nu_0, nu_1), G_10) of a row pair from its slot blocks (lane = slot, zero
// blocks on lanes 9-15): the smoother's Gram terms, one definition for every
// kernel that forms or stores them
template <typename T>
__device__ __forceinline__ void pair_gram(const cx<T> (&B)[4], cx<T>& nu, cx<T>& g10) {
  nu = grp16_sum(cx<T>{norm2_fixed(B[0]) + norm2_fixed(B[1]), norm2_fixed(B[2]) + norm2_fixed(B[3])});
  g10 = grp16_sum(cjmul_fixed(B[0], B[2]) + cjmul_fixed(B[1], B[3]));
}

template <typename T>
__global__ __launch_bounds__(256) void k_slot_gram(int nsites, const cx<T>* __restrict__ Bst, cx<T>* __restrict__ Gst) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = t >> 4, lane = t & 15;
  if (i >= nsites) return;  // whole 16-lane groups
  cx<T> B[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
  if (lane < 9) {
    const cx<T>* bp = Bst + ((size_t)i * 9 + lane) * 4;
#pragma unroll
    for (int w = 0; w < 4; ++w) B[w] = bp[w];
  }
  cx<T> nu, g10;
  pair_gram(B, nu, g10);
  if (lane == 0) {
    Gst[2 * (size_t)i] = nu;
    Gst[2 * (size_t)i + 1] = g10;
  }
}

template <typename T>
void launch_slot_gram(const FineT<T>& f, const cx<T>* Bst, cx<T>* Gst, hipStream_t s) {
  const int nsites = f.N * f.NH;
  hipLaunchKernelGGL(k_slot_gram<T>, dim3((unsigned)((nsites * 16 + 255) / 256)), dim3(256), 0, s, nsites, Bst, Gst);
}
template void launch_slot_gram<double>(const FineT<double>&, const zd*, zd*, hipStream_t);
template void launch_slot_gram<float>(const FineT<float>&, const zf*, zf*, hipStream_t);

// lam (may be NULL): per right-hand side shift, the pass then works on
// (Dhat - lam Gamma_5) x = 0 (the eigen-relaxation of the bootstrap setup,
// Sec. 3.4 / Theorem 1), Gamma_5 = +1 on spin 0 and -1 on spin 1.
// A 16-lane group (lane = stencil slot) takes one site of the colour for RB
// right-hand sides: the site's stored slot blocks, row norms and G_10 are
// read and formed once, the supports and right-hand sides of all RB are
// loaded before the first update.  Every product is contracted the same way
// whatever RB is (cmul_fixed, cjmul_fixed, norm2_fixed), so a right-hand
// side's result does not depend on how many share the group.
template <typename T, int RB>
__global__ __launch_bounds__(64) void k_kaczmarz_fine(FineT<T> f, int colour, int nsites, cx<T>* __restrict__ x,
                                                      const cx<T>* __restrict__ b, const double* __restrict__ lam,
                                                      int nrhs) {
  using C = cx<T>;
  const int lane = threadIdx.x & 15;
  // each XCD takes a contiguous range of the colour's sites, so the cache
  // lines that neighbouring sites' supports share stay in one L2
  const int t = (int)xcd_block(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 4);
  const int rbeg = blockIdx.y * RB;
  if (t >= nsites || rbeg >= nrhs) return;  // whole 16-lane groups leave together
  const size_t n = (size_t)f.N * f.NH * 2;
  int px, y;
  fine_colour_site(colour, t, f.N, px, y);
  const int i = y * f.NH + (px >> 1);
  const bool act = lane < 9;
  const int slot = act ? lane : 0;
  const int jn = hidx(px + nib(SLOT_DX2, slot) - 2, y + nib(SLOT_DY2, slot) - 2, f.N, f.NH);
  C B[2][2] = {{{0, 0}, {0, 0}}, {{0, 0}, {0, 0}}};
  if (act) {
    const C* bp = f.Bst + ((size_t)i * 9 + slot) * 4;
    B[0][0] = bp[0];
    B[0][1] = bp[1];
    B[1][0] = bp[2];
    B[1][1] = bp[3];
  }
  C x0[RB], x1[RB], b0[RB], b1[RB];
#pragma unroll
  for (int k = 0; k < RB; ++k) {
    const int r = rbeg + k;
    x0[k].x = x0[k].y = x1[k].x = x1[k].y = T(0);
    b0[k].x = b0[k].y = b1[k].x = b1[k].y = T(0);
    if (r < nrhs) {
      if (act) {
        x0[k] = x[r * n + 2 * jn];
        x1[k] = x[r * n + 2 * jn + 1];
      }
      if (b) {
        b0[k] = b[r * n + 2 * i];
        b1[k] = b[r * n + 2 * i + 1];
      }
    }
  }
  auto gram = [&](const C (&Bm)[2][2], C& nu, C& g10) {
    nu = grp16_sum(C{norm2_fixed(Bm[0][0]) + norm2_fixed(Bm[0][1]), norm2_fixed(Bm[1][0]) + norm2_fixed(Bm[1][1])});
    g10 = grp16_sum(cjmul_fixed(Bm[0][0], Bm[1][0]) + cjmul_fixed(Bm[0][1], Bm[1][1]));
  };
  C nu, g10;
  // formed here rather than read from Gst: the passes run where memory, not
  // arithmetic, bounds them, and the stored terms would add 2 entries per site
  if (!lam) gram(B, nu, g10);
#pragma unroll
  for (int k = 0; k < RB; ++k) {
    const int r = rbeg + k;
    if (r >= nrhs) break;  // uniform over the group
    C Bk[2][2] = {{B[0][0], B[0][1]}, {B[1][0], B[1][1]}};
    if (lam) {
      if (act && slot == 0) {  // slot 0 is the site itself: the diagonal 2 x 2 block
        const T l = (T)lam[r];
        Bk[0][0].x -= l;
        Bk[1][1].x += l;
      }
      gram(Bk, nu, g10);
    }
    const C r0 = grp16_sum(cmul_fixed(Bk[0][0], x0[k]) + cmul_fixed(Bk[0][1], x1[k]));
    const C r1 = grp16_sum(cmul_fixed(Bk[1][0], x0[k]) + cmul_fixed(Bk[1][1], x1[k]));
    C a0, a1;
    kz_coefs(nu, g10, b0[k] - r0, b1[k] - r1, a0, a1);
    if (act) {
      x[r * n + 2 * jn] = (x0[k] + cjmul_fixed(Bk[0][0], a0)) + cjmul_fixed(Bk[1][0], a1);
      x[r * n + 2 * jn + 1] = (x1[k] + cjmul_fixed(Bk[0][1], a0)) + cjmul_fixed(Bk[1][1], a1);
    }
  }
}

template <typename T>
void launch_kaczmarz_fine(const FineT<T>& f, int colour, int nsites, cx<T>* x, const cx<T>* b, int nrhs, hipStream_t s,
                          const double* lam) {
  if (nrhs >= 16)
    hipLaunchKernelGGL((k_kaczmarz_fine<T, 4>), dim3((nsites + 3) / 4, (nrhs + 3) / 4), dim3(64), 0, s, f, colour,
                       nsites, x, b, lam, nrhs);
  else
    hipLaunchKernelGGL((k_kaczmarz_fine<T, 1>), dim3((nsites + 3) / 4, nrhs), dim3(64), 0, s, f, colour, nsites, x, b,
                       lam, nrhs);
}
// ---------------------------------------------------------------------------
// The colour pass on right-hand-side-interleaved vectors, xi[(site*2 + s)*R + r],
// so that every support entry of a site is one contiguous run of R entries.
// The slot terms are added in the pair order of the 16-lane butterfly of
// k_kaczmarz_fine (slots 9-15 contributing +0) and every product has the same
// fixed contraction, so the result is bitwise that of k_kaczmarz_fine.
// ---------------------------------------------------------------------------
// Four lanes per (site, right-hand side): lane q = lane / 16 takes the slots
// q and q + 4 (and 8 for q = 0), the 16 lanes of a quarter are 16
// consecutive right-hand sides.  A lane forms t4[q] = (v[q] + v'[q]) +
// (v[q+4] + z) of the butterfly, with v'[0] = v[8] and v'[q] = z otherwise;
// two exchanges (quarters q ^ 2, then q ^ 1) finish the butterfly in its own
// pair order, so the sums are bitwise those of k_kaczmarz_fine.
template <typename T>
__device__ __forceinline__ cx<T> quarter_sum(cx<T> v) {
  v.x += __shfl_xor(v.x, 32, 64);
  v.y += __shfl_xor(v.y, 32, 64);
  v.x += __shfl_xor(v.x, 16, 64);
  v.y += __shfl_xor(v.y, 16, 64);
  return v;
}

template <typename T>
__global__ __launch_bounds__(64) void k_kaczmarz_fine_il(FineT<T> f, int colour, int nsites, cx<T>* __restrict__ xi,
                                                         const cx<T>* __restrict__ bi, int R) {
  using C = cx<T>;
  const int lane = threadIdx.x, q = lane >> 4;
  const int t = blockIdx.x;
  const int r = blockIdx.y * 16 + (lane & 15);
  if (t >= nsites || r >= R) return;  // the four lanes of a (site, r) leave together
  int px, y;
  fine_colour_site(colour, t, f.N, px, y);
  const int i = y * f.NH + (px >> 1);
  const C* bst = f.Bst + (size_t)i * 9 * 4;
  const int sa = q, sb = q + 4;  // this lane's slots; quarter 0 also takes slot 8
  const int ja = hidx(px + nib(SLOT_DX2, sa) - 2, y + nib(SLOT_DY2, sa) - 2, f.N, f.NH);
  const int jb = hidx(px + nib(SLOT_DX2, sb) - 2, y + nib(SLOT_DY2, sb) - 2, f.N, f.NH);
  const int j8 = hidx(px + nib(SLOT_DX2, 8) - 2, y + nib(SLOT_DY2, 8) - 2, f.N, f.NH);
  const C c00 = cmul_fixed(C{0, 0}, C{0, 0}), j00 = cjmul_fixed(C{0, 0}, C{0, 0});
  const T n00 = norm2_fixed(C{0, 0});
  const C zr = c00 + c00, zg = j00 + j00, zn = C{n00 + n00, n00 + n00};
  auto ld = [&](int j, int sp) { return xi[((size_t)j * 2 + sp) * R + r]; };
  // slot terms: rows of D x, row norms, G_10
  C B[3][4], X0[3], X1[3];
  const int js[3] = {ja, jb, j8};
  const int ss[3] = {sa, sb, 8};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int sl = ss[k];
#pragma unroll
    for (int e = 0; e < 4; ++e) B[k][e] = bst[sl * 4 + e];
    X0[k] = ld(js[k], 0);
    X1[k] = ld(js[k], 1);
  }
  C w0[3], w1[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    w0[k] = cmul_fixed(B[k][0], X0[k]) + cmul_fixed(B[k][1], X1[k]);
    w1[k] = cmul_fixed(B[k][2], X0[k]) + cmul_fixed(B[k][3], X1[k]);
  }
  const bool q0 = q == 0;
  const C r0 = quarter_sum((w0[0] + (q0 ? w0[2] : zr)) + (w0[1] + zr));
  const C r1 = quarter_sum((w1[0] + (q0 ? w1[2] : zr)) + (w1[1] + zr));
  C nu, g10;
  if (f.Gst) {  // the stored Gram terms of the row pair (the same bits)
    nu = f.Gst[2 * (size_t)i];
    g10 = f.Gst[2 * (size_t)i + 1];
  } else {
    C wn[3], wg[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      wn[k] = C{norm2_fixed(B[k][0]) + norm2_fixed(B[k][1]), norm2_fixed(B[k][2]) + norm2_fixed(B[k][3])};
      wg[k] = cjmul_fixed(B[k][0], B[k][2]) + cjmul_fixed(B[k][1], B[k][3]);
    }
    nu = quarter_sum((wn[0] + (q0 ? wn[2] : zn)) + (wn[1] + zn));
    g10 = quarter_sum((wg[0] + (q0 ? wg[2] : zg)) + (wg[1] + zg));
  }
  C b0 = {0, 0}, b1 = {0, 0};
  if (bi) {
    b0 = bi[((size_t)i * 2) * R + r];
    b1 = bi[((size_t)i * 2 + 1) * R + r];
  }
  C a0, a1;
  kz_coefs(nu, g10, b0 - r0, b1 - r1, a0, a1);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (k == 2 && !q0) break;
    xi[((size_t)js[k] * 2) * R + r] = (X0[k] + cjmul_fixed(B[k][0], a0)) + cjmul_fixed(B[k][2], a1);
    xi[((size_t)js[k] * 2 + 1) * R + r] = (X1[k] + cjmul_fixed(B[k][1], a0)) + cjmul_fixed(B[k][3], a1);
  }
}

// out[j * R + r] = in[r * n + j] (to_il) or back; 32 x 32 tiles through LDS
template <typename C>
__global__ __launch_bounds__(256) void k_transpose_rhs(const C* __restrict__ in, C* __restrict__ out, size_t n, int R,
                                                       bool to_il) {
  __shared__ C tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  const size_t j0 = (size_t)blockIdx.x * 32;
  const int r0 = blockIdx.y * 32;
  if (to_il) {
    for (int k = ty; k < 32; k += 8) {  // read rows r of [R][n] along j
      const int r = r0 + k;
      const size_t j = j0 + tx;
      if (r < R && j < n) tile[k][tx] = in[(size_t)r * n + j];
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {  // write rows j of [n][R] along r
      const size_t j = j0 + k;
      const int r = r0 + tx;
      if (r < R && j < n) out[j * R + r] = tile[tx][k];
    }
  } else {
    for (int k = ty; k < 32; k += 8) {
      const size_t j = j0 + k;
      const int r = r0 + tx;
      if (r < R && j < n) tile[tx][k] = in[j * R + r];
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
      const int r = r0 + k;
      const size_t j = j0 + tx;
      if (r < R && j < n) out[(size_t)r * n + j] = tile[k][tx];
    }
  }
}

// count sweeps on level 0 for R right-hand sides through the interleaved
// layout: x and b ([R][n]) are transposed into xi and bi, swept, and x is
// transposed back
template <typename T>
void launch_smooth_fine_il(const FineT<T>& f, int ncol, int per_colour, cx<T>* x, const cx<T>* b, cx<T>* xi,
                           cx<T>* bi, int R, int count, hipStream_t s) {
  const size_t n = (size_t)f.N * f.NH * 2;
  const dim3 tg((unsigned)((n + 31) / 32), (unsigned)((R + 31) / 32));
  hipLaunchKernelGGL((k_transpose_rhs<cx<T>>), tg, dim3(256), 0, s, x, xi, n, R, true);
  if (b) hipLaunchKernelGGL((k_transpose_rhs<cx<T>>), tg, dim3(256), 0, s, b, bi, n, R, true);
  const cx<T>* bb = b ? bi : nullptr;
  for (int it = 0; it < count; ++it)
    for (int c = 0; c < ncol; ++c)
      hipLaunchKernelGGL((k_kaczmarz_fine_il<T>), dim3(per_colour, (R + 15) / 16), dim3(64), 0, s, f, c, per_colour,
                         xi, bb, R);
  hipLaunchKernelGGL((k_transpose_rhs<cx<T>>), tg, dim3(256), 0, s, xi, x, n, R, false);
}
// ---------------------------------------------------------------------------
// One whole sweep (16 colours) per launch, blocked in LDS.
//
// In the coordinates u = (x + y)/2, v = (x - y)/2 of the even sites the colour
// is 4 (u mod 4) + (v mod 4) and the support of a row pair is the 3 x 3 box
// around its site.  The values on a tile after the sweep depend only on the
// projections of sites near it: going back one colour, the region whose
// values matter grows by the boxes of that colour's sites that touch it.  The
// plan follows that recursion from the tile backwards over the 16 colours
// (rectangles, on the host) and gives, per colour, the sites a work-group must
// project and, at the start, the region it must read (the tile plus 2 sites
// on each side in u and 14 in v for tiles starting at u = v = 1 mod 4).  A
// work-group copies that region of x into LDS, reads the slot blocks,
// right-hand sides and Gram terms of its projections into registers a few
// colours ahead, runs the 16 colours with a barrier between them and writes
// its tile.  The sweep reads xin and writes xout:
// other work-groups read a tile's old values as their halo, so the two must
// not overlap.  Each projection needed for the tile
// sees the values the colour-by-colour sweep gives it, and is evaluated with
// the same expressions as k_kaczmarz_fine (16 lanes per site, the same
// group sums and fixed contractions), so the result is bitwise that of the 16
// colour passes.  Projections near the region edge that no tile value depends
// on may see stale inputs; they only write outside the tile's dependence.
// ---------------------------------------------------------------------------
// (P xc) at spin s of even site e (half-x index) for one right-hand side:
// the 8 test-vector columns of the site's 4 x 4 aggregate, summed in order
// with fixed contractions (the prolongation kernel and the sweeps that carry
// it give the same bits)
template <typename T>
__device__ __forceinline__ cx<T> fine_prolong_entry(const FineT<T>& f, const cx<T>* __restrict__ P,
                                                    const cx<T>* __restrict__ xc, int e, int s) {
  const int cxn = f.NH / 4;
  const int y = e / f.NH, xh = e - y * f.NH;
  const int a = (y >> 2) * cxn + (xh >> 2), row = 4 * (y & 3) + (xh & 3);
  const cx<T>* Pr = P + (((size_t)a * 2 + s) * 16 + row) * 8;
  const cx<T>* xcv = xc + (size_t)a * 16 + 8 * s;
  cx<T> acc = {0, 0};
#pragma unroll
  for (int k = 0; k < 8; ++k) acc = acc + cmul_fixed(Pr[k], xcv[k]);
  return acc;
}

constexpr uint64_t SLOT_DU1 = 0x011202021ull, SLOT_DV1 = 0x102120021ull;  // (du, dv) + 1 of slot n

constexpr int FS_NT = 512;               // threads per work-group of the blocked sweep
constexpr int FS_GROUPS = FS_NT / 16;    // 16-lane groups, one projection each per step
constexpr int FS_BATCH = 16;             // 16-byte loads in flight per thread while filling LDS

// Work-group barrier for LDS only: waits for this wave's LDS accesses
// (lgkmcnt 0) but not for its global loads, which stay in flight across it
// (__syncthreads waits for every outstanding access, so the next macro-step's
// loads could not overlap the current one).  The empty asm statements keep the
// compiler from moving LDS accesses across the barrier.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);  // vmcnt 63, expcnt 7, lgkmcnt 0
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// the projections one 16-lane group makes in one colour (at most ITER), read
// from global memory (L2) fs_ahead colours before they are needed: slot
// blocks, right-hand side, stored Gram terms, and the position of the lane's
// support entry in the region (k < 0: none)
template <typename T, int ITER>
struct FsColour {
  cx<T> B[ITER][4];
  cx<T> b[ITER][2];
  cx<T> nu[ITER], g10[ITER];  // the row pair's stored Gram terms
  int e[ITER];
};
// colours read ahead: three, or one where four sets would not fit the
// registers of the FP64 form with two projections per group
template <typename T, int ITER>
constexpr int fs_ahead() {
  return (sizeof(T) == 8 && ITER == 2) ? 1 : 3;
}

template <typename T, int ITER>
__device__ __forceinline__ FsColour<T, ITER> fs_colour(const FineT<T>& f, const int (&k)[ITER], bool act, int slot,
                                                       int soff, const int* usite, const int* uloc,
                                                       const cx<T>* br, const zd* b64) {
  // reads without branches on the data (an absent projection reads
  // projection 0 and drops it), so that they stay in flight while the
  // current colours compute
  FsColour<T, ITER> r;
  const cx<T> z = {0, 0};
#pragma unroll
  for (int it = 0; it < ITER; ++it) {
    const int kq = k[it] >= 0 ? k[it] : 0;
    const size_t site = (size_t)usite[kq];
    r.e[it] = uloc[kq] + soff;
    const cx<T>* Bp = f.Bst + (site * 9 + slot) * 4;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const cx<T> v = Bp[w];
      r.B[it][w] = act ? v : z;
    }
    if (b64) {  // rounded as the conversion kernels round
      const zd v0 = b64[2 * site], v1 = b64[2 * site + 1];
      r.b[it][0] = cx<T>{(T)v0.x, (T)v0.y};
      r.b[it][1] = cx<T>{(T)v1.x, (T)v1.y};
    } else if (br) {
      r.b[it][0] = br[2 * site];
      r.b[it][1] = br[2 * site + 1];
    } else {
      r.b[it][0] = z;
      r.b[it][1] = z;
    }
    r.nu[it] = f.Gst[2 * site];
    r.g10[it] = f.Gst[2 * site + 1];
  }
  return r;
}

template <typename T, int LDSB, int ITER>
__global__ __launch_bounds__(FS_NT) void k_kaczmarz_fine_sweep(FineT<T> f, FineSweepPlan p, const cx<T>* __restrict__ xin,
                                                               cx<T>* __restrict__ xout, const cx<T>* __restrict__ b,
                                                               FineFuse<T> fz) {
  using C = cx<T>;
  constexpr int US = 2 * (int)sizeof(C) / 16;   // 16-byte units of a site's two unknowns
  __shared__ uint4 sm[LDSB / 16];
  C* X = reinterpret_cast<C*>(sm);      // region of x, [Ru][Rv][2]
  int* usite = reinterpret_cast<int*>(X + 2 * p.Ru * p.Rv);  // the projections' even-site index
  int* uloc = usite + p.nupd;                                // their position in the region
  const int tid = threadIdx.x;
  const int N = f.N, NH = f.NH;
  const int u0 = 1 + (int)(blockIdx.x % p.ntu) * p.Tu, v0 = 1 + (int)(blockIdx.x / p.ntu) * p.Tv;
  const size_t n = (size_t)N * NH * 2;
  const C* xr = xin + blockIdx.y * n;
  C* xw = xout + blockIdx.y * n;
  // b64: b comes from the FP64 copy, rounded
  const zd* b64 = fz.b64 ? fz.b64 + blockIdx.y * n : nullptr;
  const C* br = (b && !b64) ? b + blockIdx.y * n : nullptr;
  const bool xzero = fz.xzero || b64;
  auto site = [&](int u, int v) {
    const int xx = (u + v + 2 * N) % N, yy = (u - v + 2 * N) % N;
    return yy * NH + (xx >> 1);
  };
  for (int q = tid; q < p.nupd; q += FS_NT) {
    int c = 0;
    while (q >= p.first[c + 1]) ++c;
    const int k = q - p.first[c];
    const int i = p.si0[c] + 4 * (k / p.nj[c]), j = p.sj0[c] + 4 * (k % p.nj[c]);
    usite[q] = site(u0 + i, v0 + j);
    uloc[q] = (i - p.i0) * p.Rv + (j - p.j0);
  }
  // one round of loads fills the region of x (16-byte units)
  if (!xzero) {
    const int t1 = p.Ru * p.Rv * US;
    const uint4* x4 = reinterpret_cast<const uint4*>(xr);
    for (int e0 = tid; e0 < t1; e0 += FS_NT * FS_BATCH) {
      uint4 v[FS_BATCH];
#pragma unroll
      for (int u = 0; u < FS_BATCH; ++u) {
        const int e = e0 + u * FS_NT;
        v[u] = make_uint4(0, 0, 0, 0);
        if (e < t1) {
          const int q = e / US, li = q / p.Rv;
          v[u] = x4[(size_t)site(u0 + p.i0 + li, v0 + p.j0 + (q - li * p.Rv)) * US + (e - q * US)];
        }
      }
#pragma unroll
      for (int u = 0; u < FS_BATCH; ++u) {
        const int e = e0 + u * FS_NT;
        if (e < t1) sm[e] = v[u];
      }
    }
  } else {
    for (int e = tid; e < 2 * p.Ru * p.Rv; e += FS_NT) X[e] = C{0, 0};
  }
  __syncthreads();
  if (fz.P) {  // x + P xc on the region: the prolongation carried by this sweep
    const C* xcr = fz.xc + blockIdx.y * ((size_t)(NH / 4) * (N / 4) * 16);
    for (int e = tid; e < 2 * p.Ru * p.Rv; e += FS_NT) {
      const int q = e >> 1, li = q / p.Rv;
      const int st = site(u0 + p.i0 + li, v0 + p.j0 + (q - li * p.Rv));
      X[e] = X[e] + fine_prolong_entry(f, fz.P, xcr, st, e & 1);
    }
    __syncthreads();
  }
  const int g = tid >> 4, lane = tid & 15;
  const bool act = lane < 9;
  const int slot = act ? lane : 0;
  const int soff = (nib(SLOT_DU1, slot) - 1) * p.Rv + (nib(SLOT_DV1, slot) - 1);
  // the group's projections of every colour, fixed before the first step
  int kk[16][ITER];
#pragma unroll
  for (int c = 0; c < 16; ++c)
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
      const int k = p.first[c] + g + it * FS_GROUPS;
      kk[c][it] = k < p.first[c + 1] ? k : -1;
    }
  // colour c's data in ring[c % (AH + 1)], read AH colours ahead
  constexpr int AH = fs_ahead<T, ITER>();
  FsColour<T, ITER> ring[AH + 1];
#pragma unroll
  for (int c = 0; c < AH; ++c) ring[c] = fs_colour<T, ITER>(f, kk[c], act, slot, soff, usite, uloc, br, b64);
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    const FsColour<T, ITER>& cur = ring[c % (AH + 1)];
    C x0[ITER], x1[ITER];
#pragma unroll
    for (int it = 0; it < ITER; ++it) {  // the unknowns first: their reads head the LDS queue
      const C v0 = X[2 * cur.e[it]], v1 = X[2 * cur.e[it] + 1];
      x0[it] = act ? v0 : C{0, 0};
      x1[it] = act ? v1 : C{0, 0};
    }
    if (c + AH < 16)
      ring[(c + AH) % (AH + 1)] = fs_colour<T, ITER>(f, kk[c + AH < 16 ? c + AH : c], act, slot, soff, usite, uloc, br, b64);
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
      if (kk[c][it] < 0) continue;  // whole 16-lane groups
      const int e = cur.e[it];
      const C* B = cur.B[it];
      const C b0 = cur.b[it][0], b1 = cur.b[it][1];
      const C nu = cur.nu[it], g10 = cur.g10[it];
      const C r0 = grp16_sum(cmul_fixed(B[0], x0[it]) + cmul_fixed(B[1], x1[it]));
      const C r1 = grp16_sum(cmul_fixed(B[2], x0[it]) + cmul_fixed(B[3], x1[it]));
      C a0, a1;
      kz_coefs(nu, g10, b0 - r0, b1 - r1, a0, a1);
      if (act) {
        X[2 * e] = (x0[it] + cjmul_fixed(B[0], a0)) + cjmul_fixed(B[2], a1);
        X[2 * e + 1] = (x1[it] + cjmul_fixed(B[1], a0)) + cjmul_fixed(B[3], a1);
      }
    }
    // LDS only: the colours' reads from global memory stay in flight
    lds_barrier();
  }
  if (b64) {  // the tile's right-hand side, rounded, for the sweeps that follow
    C* bo = fz.b_out + blockIdx.y * n;
    for (int e = tid; e < p.Tu * p.Tv * 2; e += FS_NT) {
      const int q = e >> 1, ti = q / p.Tv, tj = q - ti * p.Tv;
      const size_t at = 2 * (size_t)site(u0 + ti, v0 + tj) + (e & 1);
      const zd v = b64[at];
      bo[at] = C{(T)v.x, (T)v.y};
    }
  }
  if (fz.x64) {
    zd* xo = fz.x64 + blockIdx.y * n;
    for (int e = tid; e < p.Tu * p.Tv * 2; e += FS_NT) {
      const int q = e >> 1, ti = q / p.Tv, tj = q - ti * p.Tv;
      const int l = (ti - p.i0) * p.Rv + (tj - p.j0);
      const C v = X[2 * l + (e & 1)];
      xo[2 * (size_t)site(u0 + ti, v0 + tj) + (e & 1)] = zd{(double)v.x, (double)v.y};
    }
    return;
  }
  uint4* xw4 = reinterpret_cast<uint4*>(xw);
  for (int e = tid; e < p.Tu * p.Tv * US; e += FS_NT) {
    const int q = e / US, ti = q / p.Tv, tj = q - ti * p.Tv;
    const int l = (ti - p.i0) * p.Rv + (tj - p.j0);
    xw4[(size_t)site(u0 + ti, v0 + tj) * US + (e - q * US)] = sm[l * US + (e - q * US)];
  }
}

// The same sweep for larger lattices, streaming: LDS holds the region of x,
// one colour's slot blocks and right-hand sides, and the projection tables.
// While a colour is projected, the next colour's slot blocks and right-hand
// sides are loaded into registers; after the colour's barrier they are
// stored to LDS, and a second barrier makes them visible.  Larger tiles fit
// than in the form above (1.3-1.6 projections per tile site), so each slot
// block is read about 1.4 times per sweep instead of the 16 colour passes'
// 9-fold touch of every x entry.  1024 threads: 64 groups of 16 lanes.
constexpr int FSS_NT = 1024, FSS_GROUPS = FSS_NT / 16;
// staged 16-byte loads per thread at most (more would spill FP64 registers)
template <typename T>
constexpr int FSS_SB_MAX = sizeof(T) == 8 ? 4 : 8;

template <typename T>
static size_t fine_sweep_lds_s(const FineSweepPlan& p, int maxcnt) {
  return (size_t)(2 * p.Ru * p.Rv + 40 * maxcnt) * sizeof(cx<T>) + 8 * (size_t)p.nupd;
}

template <typename T, int LDSB, int ITER, int SB>
__global__ __launch_bounds__(FSS_NT) void k_kaczmarz_fine_sweep_s(FineT<T> f, FineSweepPlan p, int maxcnt,
                                                                  const cx<T>* __restrict__ xin, cx<T>* __restrict__ xout,
                                                                  const cx<T>* __restrict__ b) {
  using C = cx<T>;
  constexpr int UB = 36 * (int)sizeof(C) / 16;  // 16-byte units of a site's slot blocks
  constexpr int US = 2 * (int)sizeof(C) / 16;   // 16-byte units of a site's two unknowns
  __shared__ uint4 sm[LDSB / 16];
  C* X = reinterpret_cast<C*>(sm);              // region of x, [Ru][Rv][2]
  uint4* Bu = sm + p.Ru * p.Rv * US;            // the colour's slot blocks, [maxcnt][36]
  uint4* bu = Bu + maxcnt * UB;                 // the colour's right-hand sides, [maxcnt][2]
  uint4* gu = bu + maxcnt * US;                 // the colour's stored Gram terms, [maxcnt][2]
  int* usite = reinterpret_cast<int*>(gu + maxcnt * US);  // even-site index of every projection
  int* uloc = usite + p.nupd;                             // its position in the region
  const int tid = threadIdx.x;
  const int N = f.N, NH = f.NH;
  const int u0 = 1 + (int)(blockIdx.x % p.ntu) * p.Tu, v0 = 1 + (int)(blockIdx.x / p.ntu) * p.Tv;
  const size_t n = (size_t)N * NH * 2;
  const C* xr = xin + blockIdx.y * n;
  C* xw = xout + blockIdx.y * n;
  const C* br = b ? b + blockIdx.y * n : nullptr;
  const int ub = UB + (br ? US : 0) + US;  // units per projection
  auto site = [&](int u, int v) {
    const int xx = (u + v + 2 * N) % N, yy = (u - v + 2 * N) % N;
    return yy * NH + (xx >> 1);
  };
  for (int q = tid; q < p.nupd; q += FSS_NT) {
    int c = 0;
    while (q >= p.first[c + 1]) ++c;
    const int k = q - p.first[c];
    const int i = p.si0[c] + 4 * (k / p.nj[c]), j = p.sj0[c] + 4 * (k % p.nj[c]);
    usite[q] = site(u0 + i, v0 + j);
    uloc[q] = (i - p.i0) * p.Rv + (j - p.j0);
  }
  {
    const int t1 = p.Ru * p.Rv * US;
    const uint4* x4 = reinterpret_cast<const uint4*>(xr);
    for (int e0 = tid; e0 < t1; e0 += FSS_NT * 4) {
      uint4 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + u * FSS_NT;
        v[u] = make_uint4(0, 0, 0, 0);
        if (e < t1) {
          const int q = e / US, li = q / p.Rv;
          v[u] = x4[(size_t)site(u0 + p.i0 + li, v0 + p.j0 + (q - li * p.Rv)) * US + (e - q * US)];
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + u * FSS_NT;
        if (e < t1) sm[e] = v[u];
      }
    }
  }
  __syncthreads();
  // colour c's data in 16-byte units: [0, cnt UB) slot blocks, then the
  // Gram terms, then the right-hand sides (if any); loaded into stg[],
  // stored to Bu / gu / bu
  const uint4* B4 = reinterpret_cast<const uint4*>(f.Bst);
  const uint4* b4 = reinterpret_cast<const uint4*>(br);
  const uint4* G4 = reinterpret_cast<const uint4*>(f.Gst);
  uint4 stg[SB];
  auto stage = [&](int c) {
    const int f0 = p.first[c], cnt = p.first[c + 1] - f0, nB = cnt * UB, nG = nB + cnt * US, tot = cnt * ub;
#pragma unroll
    for (int u = 0; u < SB; ++u) {
      const int e = tid + u * FSS_NT;
      stg[u] = make_uint4(0, 0, 0, 0);
      if (e < tot) {
        const uint4* src;
        size_t idx;
        if (e < nB) {
          const int q = e / UB;
          src = B4;
          idx = (size_t)usite[f0 + q] * UB + (e - q * UB);
        } else if (e < nG) {
          const int q = (e - nB) / US;
          src = G4;
          idx = (size_t)usite[f0 + q] * US + (e - nB - q * US);
        } else {
          const int q = (e - nG) / US;
          src = b4;
          idx = (size_t)usite[f0 + q] * US + (e - nG - q * US);
        }
        stg[u] = src[idx];
      }
    }
  };
  auto commit = [&](int c) {
    const int cnt = p.first[c + 1] - p.first[c], nB = cnt * UB, nG = nB + cnt * US, tot = cnt * ub;
#pragma unroll
    for (int u = 0; u < SB; ++u) {
      const int e = tid + u * FSS_NT;
      if (e < tot) {
        if (e < nB) Bu[e] = stg[u];
        else if (e < nG) gu[e - nB] = stg[u];
        else bu[e - nG] = stg[u];
      }
    }
  };
  stage(0);
  commit(0);
  __syncthreads();
  const int g = tid >> 4, lane = tid & 15;
  const bool act = lane < 9;
  const int slot = act ? lane : 0;
  const int soff = (nib(SLOT_DU1, slot) - 1) * p.Rv + (nib(SLOT_DV1, slot) - 1);
  const C* BC = reinterpret_cast<const C*>(Bu) + slot * 4;
  const C* bC = reinterpret_cast<const C*>(bu);
  const C* gC = reinterpret_cast<const C*>(gu);
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    if (c < 15) stage(c + 1);  // in flight while colour c is projected
    const int f0 = p.first[c], cnt = p.first[c + 1] - f0;
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
      const int kl = g + it * FSS_GROUPS;
      if (kl >= cnt) continue;  // whole 16-lane groups
      const int e = uloc[f0 + kl] + soff;
      C B[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
      C x0 = {0, 0}, x1 = {0, 0}, b0 = {0, 0}, b1 = {0, 0};
      if (act) {
#pragma unroll
        for (int w = 0; w < 4; ++w) B[w] = BC[kl * 36 + w];
        x0 = X[2 * e];
        x1 = X[2 * e + 1];
      }
      if (br) {
        b0 = bC[2 * kl];
        b1 = bC[2 * kl + 1];
      }
      const C nu = gC[2 * kl], g10 = gC[2 * kl + 1];
      const C r0 = grp16_sum(cmul_fixed(B[0], x0) + cmul_fixed(B[1], x1));
      const C r1 = grp16_sum(cmul_fixed(B[2], x0) + cmul_fixed(B[3], x1));
      C a0, a1;
      kz_coefs(nu, g10, b0 - r0, b1 - r1, a0, a1);
      if (act) {
        X[2 * e] = (x0 + cjmul_fixed(B[0], a0)) + cjmul_fixed(B[2], a1);
        X[2 * e + 1] = (x1 + cjmul_fixed(B[1], a0)) + cjmul_fixed(B[3], a1);
      }
    }
    __syncthreads();
    if (c < 15) {
      commit(c + 1);
      __syncthreads();
    }
  }
  uint4* xw4 = reinterpret_cast<uint4*>(xw);
  for (int e = tid; e < p.Tu * p.Tv * US; e += FSS_NT) {
    const int q = e / US, ti = q / p.Tv, tj = q - ti * p.Tv;
    const int l = (ti - p.i0) * p.Rv + (tj - p.j0);
    xw4[(size_t)site(u0 + ti, v0 + tj) * US + (e - q * US)] = sm[l * US + (e - q * US)];
  }
}

// ---------------------------------------------------------------------------
// The sweep blocked in LDS for large lattices: a pipelined march along v.
// A work-group owns a tile of FP_TU x Tv even sites (u, v) and the same
// dependence region as the blocked sweeps (fine_sweep_plan), but it never
// holds the whole region: it marches down v with a ring of FP_W columns of x
// in LDS.  In the colour order the dependence between two projections of
// colours c' < c that share an unknown spans |dv| <= 2; colour c projects
// column sj0[c] + 4 k at macro-step k + c, so at any macro-step the active
// columns of the 16 colours lie 3 apart (their 3 x 3 supports are disjoint)
// and every projection follows those it depends on: all 16 colours run
// together, one barrier per macro-step, and the result is bitwise that of the
// colour-by-colour sweep (the host checks the schedule and the ring; a CPU
// replay pins it).  Every (colour, row) pair of the plan has a four-lane
// group of its own, whose site moves by 4 in v per macro-step; it reads its
// stored slot blocks and Gram terms one macro-step ahead.  Four lanes per projection,
// lane q taking the slots q, q + 4 (and 8 for q = 0) and finishing the
// 16-lane butterfly with two quad exchanges, as k_kaczmarz_fine_il does.
// The next macro-step's columns are read while the current one projects; a
// column whose ring slot is taken again is written out first if it belongs
// to the tile.  xin and xout must not overlap.
// ---------------------------------------------------------------------------
constexpr int FP_TU = 16;               // tile extent in u
constexpr int FP_W = 48;                // ring columns
constexpr int FP_RU_MAX = 24;           // region extent in u the ring holds
constexpr int FP_NT = 320;              // threads: 80 four-lane groups
constexpr int FP_GROUPS = FP_NT / 4;

struct FinePipePlan {
  int Tu, Tv, ntu, ntv, i0, j0, Ru, Rv, M, A;
  int si0[16], sj0[16], ni[16], nj[16], off[16];
};

// sum over the 4 lanes of a quad: partner q ^ 2, then q ^ 1 (the last two
// steps of the 16-lane butterfly, in its pair order)
template <typename T>
__device__ __forceinline__ cx<T> quad_sum(cx<T> v) {
  v.x += dpp_mov<DPP_QUAD_XOR2>(v.x);
  v.y += dpp_mov<DPP_QUAD_XOR2>(v.y);
  v.x += dpp_mov<DPP_QUAD_XOR1>(v.x);
  v.y += dpp_mov<DPP_QUAD_XOR1>(v.y);
  return v;
}

// wrap a lattice coordinate that is at most one period off
__device__ __forceinline__ int wrap1(int a, int N) { return a < 0 ? a + N : (a >= N ? a - N : a); }

template <typename T>
__global__ __launch_bounds__(FP_NT) void k_kaczmarz_fine_pipe(FineT<T> f, FinePipePlan p, const cx<T>* __restrict__ xin,
                                                              cx<T>* __restrict__ xout, const cx<T>* __restrict__ b) {
  using C = cx<T>;
  constexpr int RP = FP_W * FP_RU_MAX;  // ring positions: position = column slot * FP_RU_MAX + row
  __shared__ C X[RP * 2];   // unknowns
  __shared__ C BR[RP * 2];  // right-hand sides
  const int tid = threadIdx.x;
  const int N = f.N, NH = f.NH;
  const int tile = (int)xcd_block(blockIdx.x, gridDim.x);
  const int u0 = 1 + (tile % p.ntu) * p.Tu, v0 = 1 + (tile / p.ntu) * p.Tv;
  const size_t n = (size_t)N * NH * 2;
  const C* __restrict__ xr = xin + blockIdx.y * n;
  C* __restrict__ xw = xout + blockIdx.y * n;
  const C* __restrict__ br = b ? b + blockIdx.y * n : nullptr;
  const int Ru = p.Ru, Rv = p.Rv;
  // lattice coordinates of region position (ri, cj)
  auto lxy = [&](int ri, int cj, int& xx, int& yy) {
    const int u = u0 + p.i0 + ri, v = v0 + p.j0 + cj;
    xx = ((u + v) % N + N) % N;
    yy = ((u - v) % N + N) % N;
  };
  // columns brought in at macro-step m (m >= 1): [4m + A - j0, +4); at m = 0 every column below 4 + A - j0
  const int col0_hi = min(Rv, 4 + p.A - p.j0);
  // prologue: the columns of macro-step 0 (4 entries per position: 2 unknowns, 2 right-hand sides)
  for (int e = tid; e < col0_hi * Ru * 4; e += FP_NT) {
    const int w = e & 3, qq = e >> 2, cj = qq / Ru, ri = qq - cj * Ru;
    int xx, yy;
    lxy(ri, cj, xx, yy);
    const size_t s2 = 2 * ((size_t)yy * NH + (xx >> 1));
    const int at = (cj % FP_W) * FP_RU_MAX + ri;
    if (w < 2) X[at * 2 + w] = xr[s2 + w];
    else BR[at * 2 + (w - 2)] = br ? br[s2 + (w - 2)] : C{0, 0};
  }
  // The entries this thread brings in at every macro-step m >= 1: entry e =
  // tid + k FP_NT of the 4-column block, column 4m + A - j0 + dc, row ri.  Its
  // lattice coordinates move by (+4, -4) per macro-step.
  constexpr int PF = (4 * FP_RU_MAX * 4 + FP_NT - 1) / FP_NT;
  int ew[PF], eri[PF], edc[PF], ex[PF], ey[PF];
#pragma unroll
  for (int k = 0; k < PF; ++k) {
    const int e = tid + k * FP_NT, qq = e >> 2;
    ew[k] = e & 3;
    edc[k] = qq / Ru;
    eri[k] = qq - edc[k] * Ru;
    if (edc[k] >= 4) edc[k] = 1 << 20;  // beyond the block: never loaded
    lxy(eri[k], 4 + p.A - p.j0 + edc[k], ex[k], ey[k]);  // its position at macro-step 1
  }
  // The group's projection: a fixed (colour, row) pair of the plan, whose
  // column moves by 4 per macro-step; its stored slot blocks and Gram terms
  // are read one macro-step ahead.
  const int gid = tid >> 2, q = tid & 3;
  const bool q0 = q == 0;
  int gsi = 0, gsj = 0, gnj = 0, goff = 1 << 20, gr = -1;
  {
    int acc = 0;
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      if (gr < 0 && gid < acc + p.ni[c]) {
        gr = gid - acc;
        gsi = p.si0[c];
        gsj = p.sj0[c];
        gnj = p.nj[c];
        goff = p.off[c];
      }
      acc += p.ni[c];
    }
  }
  const int gri = gsi + 4 * gr - p.i0;  // the group's row in the region
  int gx = 0, gy = 0;                   // lattice coordinates of its site at its first macro-step
  if (gr >= 0) lxy(gri, gsj - p.j0, gx, gy);
  struct Stored {
    C B[3][4];
    C nu, g10;
  };
  auto read_stored = [&](int xx, int yy, Stored& S) {
    const size_t ih = (size_t)yy * NH + (xx >> 1);
    const C* bst = f.Bst + ih * 9 * 4;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int sl = k == 0 ? q : (k == 1 ? q + 4 : (q0 ? 8 : 0));
#pragma unroll
      for (int w = 0; w < 4; ++w) S.B[k][w] = bst[sl * 4 + w];
    }
    S.nu = f.Gst[2 * ih];
    S.g10 = f.Gst[2 * ih + 1];
  };
  Stored cur, nxt;
  if (gr >= 0 && goff == 0) read_stored(gx, gy, cur);
  __syncthreads();
  const C c00 = cmul_fixed(C{0, 0}, C{0, 0});
  const C zr = c00 + c00;
  for (int m = 0; m < p.M; ++m) {
    // the next macro-step's columns and the group's next projection data,
    // in flight while this macro-step projects
    const int nc0 = 4 * (m + 1) + p.A - p.j0, nc1 = (m + 1 < p.M) ? min(Rv, nc0 + 4) : nc0;
    C pre[PF];
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      pre[k] = C{0, 0};
      if (m > 0) {  // coordinates of macro-step m + 1
        ex[k] = wrap1(ex[k] + 4, N);
        ey[k] = wrap1(ey[k] - 4, N);
      }
      if (nc0 + edc[k] < nc1) {
        const size_t s2 = 2 * ((size_t)ey[k] * NH + (ex[k] >> 1));
        if (ew[k] < 2) pre[k] = xr[s2 + ew[k]];
        else if (br) pre[k] = br[s2 + (ew[k] - 2)];
      }
    }
    const int kg = m - goff;  // the group's step along its columns
    const bool act = gr >= 0 && kg >= 0 && kg < gnj;
    const bool act_next = gr >= 0 && kg + 1 >= 0 && kg + 1 < gnj;
    int nx = gx, ny = gy;  // its site at macro-step m + 1
    if (kg + 1 >= 1) {
      nx = wrap1(gx + 4, N);
      ny = wrap1(gy - 4, N);
    }
    if (act_next) read_stored(nx, ny, nxt);
    if (act) {
      const int cj0 = gsj + 4 * kg - p.j0;
      const int site = (cj0 % FP_W) * FP_RU_MAX + gri;
      C X0[3], X1[3];
      int pos[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const int sl = k == 0 ? q : (k == 1 ? q + 4 : (q0 ? 8 : 0));
        const int ri = gri + nib(SLOT_DU1, sl) - 1, cj = cj0 + nib(SLOT_DV1, sl) - 1;
        pos[k] = (cj % FP_W) * FP_RU_MAX + ri;
        X0[k] = X[pos[k] * 2];
        X1[k] = X[pos[k] * 2 + 1];
      }
      C w0[3], w1[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        w0[k] = cmul_fixed(cur.B[k][0], X0[k]) + cmul_fixed(cur.B[k][1], X1[k]);
        w1[k] = cmul_fixed(cur.B[k][2], X0[k]) + cmul_fixed(cur.B[k][3], X1[k]);
      }
      const C r0 = quad_sum((w0[0] + (q0 ? w0[2] : zr)) + (w0[1] + zr));
      const C r1 = quad_sum((w1[0] + (q0 ? w1[2] : zr)) + (w1[1] + zr));
      const C b0 = BR[site * 2], b1 = BR[site * 2 + 1];
      const C nu = cur.nu, g10 = cur.g10;
      C a0, a1;
      kz_coefs(nu, g10, b0 - r0, b1 - r1, a0, a1);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        if (k < 2 || q0) {
          X[pos[k] * 2] = (X0[k] + cjmul_fixed(cur.B[k][0], a0)) + cjmul_fixed(cur.B[k][2], a1);
          X[pos[k] * 2 + 1] = (X1[k] + cjmul_fixed(cur.B[k][1], a0)) + cjmul_fixed(cur.B[k][3], a1);
        }
      }
    }
    if (kg + 1 >= 1) {
      gx = nx;
      gy = ny;
    }
    lds_barrier();
    // ring slots taken by the next columns: write their old column out if it
    // belongs to the tile (every projection reading it has run), then store
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      const int cj = nc0 + edc[k];
      if (cj < nc1) {
        const int at = (cj % FP_W) * FP_RU_MAX + eri[k];
        if (ew[k] < 2) {
          const int old = cj - FP_W, io = eri[k] + p.i0, jo = old + p.j0;
          if (old >= 0 && io >= 0 && io < p.Tu && jo >= 0 && jo < p.Tv) {
            const int ox = wrap1(ex[k] - FP_W, N), oy = wrap1(ey[k] + FP_W, N);
            xw[2 * ((size_t)oy * NH + (ox >> 1)) + ew[k]] = X[at * 2 + ew[k]];
          }
          X[at * 2 + ew[k]] = pre[k];
        } else {
          BR[at * 2 + (ew[k] - 2)] = pre[k];
        }
      }
    }
    lds_barrier();
    if (act_next) cur = nxt;
  }
  // the tile's columns still in the ring
  const int c0 = max(0, Rv - FP_W);
  for (int e = tid; e < (Rv - c0) * Ru * 2; e += FP_NT) {
    const int sp = e & 1, qq = e >> 1, cj = c0 + qq / Ru, ri = qq - (qq / Ru) * Ru;
    const int i = ri + p.i0, j = cj + p.j0;
    if (i >= 0 && i < p.Tu && j >= 0 && j < p.Tv) {
      int xx, yy;
      lxy(ri, cj, xx, yy);
      xw[2 * ((size_t)yy * NH + (xx >> 1)) + sp] = X[((cj % FP_W) * FP_RU_MAX + ri) * 2 + sp];
    }
  }
}

// The dependence recursion for a Tu x Tv tile whose origin has u = v = 1 mod 4
// (coordinates relative to the tile origin).  False if a projection count
// exceeds the table or the region would meet itself across the torus.
static bool fine_sweep_plan(int N, int Tu, int Tv, FineSweepPlan& p, int max_cnt = 2 * FS_GROUPS) {
  auto m4 = [](int a) { return ((a % 4) + 4) % 4; };
  int i0 = 0, i1 = Tu - 1, j0 = 0, j1 = Tv - 1;
  int cnt[16];
  for (int c = 15; c >= 0; --c) {
    const int a = c >> 2, bb = c & 3;
    const int lo_i = i0 - 1, hi_i = i1 + 1, lo_j = j0 - 1, hi_j = j1 + 1;
    const int si0 = lo_i + m4(a - 1 - lo_i), sj0 = lo_j + m4(bb - 1 - lo_j);
    p.si0[c] = si0;
    p.sj0[c] = sj0;
    if (si0 > hi_i || sj0 > hi_j) {
      cnt[c] = 0;
      p.nj[c] = 1;
      continue;
    }
    const int ni = (hi_i - si0) / 4 + 1, nj = (hi_j - sj0) / 4 + 1;
    cnt[c] = ni * nj;
    p.nj[c] = nj;
    i0 = std::min(i0, si0 - 1);
    i1 = std::max(i1, si0 + 4 * (ni - 1) + 1);
    j0 = std::min(j0, sj0 - 1);
    j1 = std::max(j1, sj0 + 4 * (nj - 1) + 1);
  }
  p.Tu = Tu;
  p.Tv = Tv;
  p.ntu = N / Tu;
  p.ntv = (N / 2) / Tv;
  p.i0 = i0;
  p.j0 = j0;
  p.Ru = i1 - i0 + 1;
  p.Rv = j1 - j0 + 1;
  p.first[0] = 0;
  for (int c = 0; c < 16; ++c) p.first[c + 1] = p.first[c] + cnt[c];
  p.nupd = p.first[16];
  for (int c = 0; c < 16; ++c)
    if (cnt[c] > max_cnt) return false;  // projection steps per group and colour are bounded
  return p.Ru <= N && p.Rv <= N && (2 * p.Ru <= N || 2 * p.Rv <= N);
}

template <typename T>
static size_t fine_sweep_lds(const FineSweepPlan& p) {
  return (size_t)(2 * p.Ru * p.Rv + 40 * p.nupd) * sizeof(cx<T>) + 8 * (size_t)p.nupd;
}

constexpr int FS_LDS_TINY = 40960, FS_LDS_SMALL = 81920, FS_LDS_LARGE = 163840;

// The tile for an N x N lattice and nrhs right-hand sides: the fewest
// projections per tile site among the tiles that give at least 256
// work-groups (one per compute unit), else the most work-groups.  Measured on
// MI355X (FP32, one right-hand side): 128^2 4 x 8, 256^2 4 x 32, 512^2 8 x 32.
template <typename T>
bool fine_sweep_choose(int N, int nrhs, FineSweepPlan& best) {
  if (N % 8 != 0 || N < 64) return false;
  bool found = false;
  double best_red = 0;
  long best_wg = 0;
  for (int Tu : {4, 8, 16, 32})
    for (int Tv : {8, 16, 32, 64, 128}) {
      if (N % Tu != 0 || (N / 2) % Tv != 0) continue;
      FineSweepPlan p;
      if (!fine_sweep_plan(N, Tu, Tv, p)) continue;
      if (fine_sweep_lds<T>(p) > (size_t)FS_LDS_LARGE) continue;
      const long wg = (long)p.ntu * p.ntv * nrhs;
      const double red = (double)p.nupd / (Tu * Tv);
      bool better;
      if (!found) better = true;
      else if (wg >= 256 && best_wg >= 256) better = red < best_red;
      else better = wg > best_wg || (wg == best_wg && red < best_red);
      if (better) {
        best = p;
        best_red = red;
        best_wg = wg;
        found = true;
      }
    }
  return found;
}

// The blocked sweep pays for its redundant projections and its per-colour
// barriers with 15 fewer launches; measured on MI355X it is the faster form
// while x is small (FP32: 1.6-2.8x at 64^2-256^2 with one right-hand side,
// even at 512^2 or 256^2 x 4; FP64: 1.9x at 128^2, even at 256^2) and the
// slower one beyond, where the colour passes stream at memory bandwidth.
constexpr size_t FS_MAX_X_BYTES = size_t(1) << 20;

// The streaming form is bound by its arithmetic (16-lane groups, 16 colour
// steps), not by memory; measured on MI355X it beats the colour passes up to
// N^2 R = 2^20 entries of x in FP32 (512^2: 41 against 56 us per sweep,
// 1024^2: 95 against 115, 256^2 x 8: 57 against 69) and 2^18 in FP64 (512^2:
// 63 against 72), and loses beyond (FP32 2048^2: 415 against 390; FP64
// 1024^2: 270 against 204), where the passes stream at memory bandwidth.
template <typename T>
constexpr size_t FSS_MAX_ENTRIES = sizeof(T) == 8 ? size_t(1) << 18 : size_t(1) << 20;

// The streaming form's tile: the fewest projections per tile site among the
// tiles whose LDS fits, whose colours need at most 4 steps of the 64 groups
// and 8 staged loads per thread, preferring at least 256 work-groups.
template <typename T>
bool fine_sweep_choose_s(int N, int nrhs, FineSweepPlan& best, int& best_maxcnt) {
  if (N % 8 != 0 || N < 64) return false;
  constexpr int UB = 36 * (int)sizeof(cx<T>) / 16, US = 2 * (int)sizeof(cx<T>) / 16;
  bool found = false;
  double best_red = 0;
  long best_wg = 0;
  for (int Tu : {4, 8, 16, 32})
    for (int Tv : {8, 16, 32, 64, 128}) {
      if (N % Tu != 0 || (N / 2) % Tv != 0) continue;
      FineSweepPlan p;
      if (!fine_sweep_plan(N, Tu, Tv, p, 4 * FSS_GROUPS)) continue;
      int maxcnt = 0;
      for (int c = 0; c < 16; ++c) maxcnt = std::max(maxcnt, p.first[c + 1] - p.first[c]);
      if (fine_sweep_lds_s<T>(p, maxcnt) > (size_t)FS_LDS_LARGE || maxcnt * (UB + 2 * US) > FSS_SB_MAX<T> * FSS_NT)
        continue;
      const long wg = (long)p.ntu * p.ntv * nrhs;
      const double red = (double)p.nupd / (Tu * Tv);
      bool better;
      if (!found) better = true;
      else if (wg >= 256 && best_wg >= 256) better = red < best_red;
      else better = wg > best_wg || (wg == best_wg && red < best_red);
      if (better) {
        best = p;
        best_maxcnt = maxcnt;
        best_red = red;
        best_wg = wg;
        found = true;
      }
    }
  return found;
}

// The pipelined sweep's plan for FP_TU x Tv tiles: the dependence rectangles
// of fine_sweep_plan, colour c at macro-step offset c (the schedule the
// kernel assumes), checked here pair by pair: every two projections whose
// supports share an unknown must run in colour order, and no two projections
// of one macro-step may share one.  The ring: column j is read at macro-step
// max(0, floor((j - A) / 4)), which must come no later than its first use,
// and its slot is taken again by column j + FP_W no earlier than the
// macro-step after its last use.  False if no A passes or the region does not
// fit the ring's rows.
static bool fine_pipe_plan(int N, int Tv, FinePipePlan& q, FineSweepPlan& p) {
  if (N % FP_TU != 0 || (N / 2) % Tv != 0 || Tv % 4 != 0) return false;
  if (!fine_sweep_plan(N, FP_TU, Tv, p, 1 << 30)) return false;
  if (p.Ru > FP_RU_MAX) return false;
  q.Tu = p.Tu; q.Tv = p.Tv; q.ntu = p.ntu; q.ntv = p.ntv;
  q.i0 = p.i0; q.j0 = p.j0; q.Ru = p.Ru; q.Rv = p.Rv;
  q.M = 0;
  for (int c = 0; c < 16; ++c) {
    q.si0[c] = p.si0[c];
    q.sj0[c] = p.sj0[c];
    q.nj[c] = p.nj[c];
    q.ni[c] = p.nj[c] > 0 ? (p.first[c + 1] - p.first[c]) / p.nj[c] : 0;
    q.off[c] = c;
    if (q.ni[c] > 0) q.M = std::max(q.M, c + q.nj[c]);
  }
  {  // the kernel gives each (colour, row) pair of the plan a four-lane group of its own
    int groups = 0;
    for (int c = 0; c < 16; ++c) groups += q.ni[c];
    if (groups > FP_GROUPS) return false;
  }
  // dependences: colours c' < c, columns j' and j within 2 of each other
  for (int c = 0; c < 16; ++c)
    for (int cp = 0; cp < c; ++cp) {
      if (!q.ni[c] || !q.ni[cp]) continue;
      for (int k = 0; k < q.nj[c]; ++k)
        for (int kp = 0; kp < q.nj[cp]; ++kp) {
          const int dj = (q.sj0[c] + 4 * k) - (q.sj0[cp] + 4 * kp);
          if (dj >= -2 && dj <= 2 && !(kp + q.off[cp] < k + q.off[c])) return false;
        }
    }
  // first and last macro-step each region column is read or written
  std::vector<int> first(p.Rv, 1 << 30), last(p.Rv, -1);
  for (int c = 0; c < 16; ++c)
    for (int k = 0; k < q.nj[c] && q.ni[c]; ++k)
      for (int dj = -1; dj <= 1; ++dj) {
        const int cj = q.sj0[c] + 4 * k + dj - p.j0;
        if (cj < 0 || cj >= p.Rv) return false;
        first[cj] = std::min(first[cj], k + q.off[c]);
        last[cj] = std::max(last[cj], k + q.off[c]);
      }
  auto floor4 = [](int a) { return a >= 0 ? a / 4 : -((-a + 3) / 4); };
  for (int A = -64; A <= 64; ++A) {
    bool ok = 4 + A - p.j0 >= 0;  // the kernel's columns of macro-step m >= 1 are 4m + A - j0 + (0..3) >= 0
    for (int cj = 0; cj < p.Rv && ok; ++cj) {
      const int j = cj + p.j0, sl = std::max(0, floor4(j - A));
      if (first[cj] < (1 << 30) && sl > first[cj]) ok = false;
      if (cj + FP_W < p.Rv) {
        const int sl2 = std::max(0, floor4(j + FP_W - A));
        if (sl2 <= last[cj] || sl2 < 1) ok = false;
      }
    }
    if (ok) {
      q.A = A;
      return true;
    }
  }
  return false;
}

// The pipelined sweep's tile for an N x N lattice: FP_TU in u and, along v,
// the tile with the fewest projections per tile site among those giving at
// least 512 work-groups (else the most work-groups).
static bool fine_pipe_choose(int N, int nrhs, FinePipePlan& best, FineSweepPlan& best_p) {
  bool found = false;
  double best_red = 0;
  long best_wg = 0;
  for (int Tv : {32, 64, 128, 256, 512}) {
    FinePipePlan q;
    FineSweepPlan p;
    if (!fine_pipe_plan(N, Tv, q, p)) continue;
    long nproj = 0;
    for (int c = 0; c < 16; ++c) nproj += (long)q.ni[c] * q.nj[c];
    const long wg = (long)q.ntu * q.ntv * nrhs;
    const double red = (double)nproj / (q.Tu * q.Tv);
    bool better;
    if (!found) better = true;
    else if (wg >= 512 && best_wg >= 512) better = red < best_red;
    else better = wg > best_wg || (wg == best_wg && red < best_red);
    if (better) {
      best = q;
      best_p = p;
      best_red = red;
      best_wg = wg;
      found = true;
    }
  }
  return found;
}

// 0: no blocked sweep, 1: LDS-resident form, 2: streaming form, 3: pipelined
// march along v (beyond the streaming form's sizes)
template <typename T>
static int fine_sweep_cached_plan(int N, int nrhs, FineSweepPlan& out, int& maxcnt, FinePipePlan* pipe = nullptr) {
  struct Cached {
    int N = -1, nrhs = -1, mode = 0, maxcnt = 0;
    FineSweepPlan p;
    FinePipePlan q;
  };
  thread_local Cached cache;
  if (cache.N != N || cache.nrhs != nrhs) {
    cache.N = N;
    cache.nrhs = nrhs;
    cache.mode = 0;
    const size_t entries = (size_t)N * N * nrhs;
    if (entries * sizeof(cx<T>) <= FS_MAX_X_BYTES && fine_sweep_choose<T>(N, nrhs, cache.p))
      cache.mode = 1;
    else if (entries <= FSS_MAX_ENTRIES<T> && fine_sweep_choose_s<T>(N, nrhs, cache.p, cache.maxcnt))
      cache.mode = 2;
    else if (fine_pipe_choose(N, nrhs, cache.q, cache.p))
      cache.mode = 3;
  }
  out = cache.p;
  maxcnt = cache.maxcnt;
  if (pipe) *pipe = cache.q;
  return cache.mode;
}

template <typename T>
bool fine_sweep_applies(const FineT<T>& f, int nrhs) {
  FineSweepPlan p;
  int maxcnt;
  if (!f.Bst || !f.Gst || nrhs < 1 || nrhs > 65535) return false;
  return fine_sweep_cached_plan<T>(f.N, nrhs, p, maxcnt) != 0;
}

template <typename T>
bool fine_sweep_fusable(const FineT<T>& f, int nrhs) {
  FineSweepPlan p;
  int maxcnt;
  if (!f.Bst || !f.Gst || nrhs < 1 || nrhs > 65535) return false;
  return fine_sweep_cached_plan<T>(f.N, nrhs, p, maxcnt) == 1;
}

template <typename T>
bool launch_fine_sweep(const FineT<T>& f, const cx<T>* xin, cx<T>* xout, const cx<T>* b, int nrhs, hipStream_t s,
                       const FineFuse<T>& fz) {
  FineSweepPlan p;
  FinePipePlan q;
  int maxcnt = 0;
  const int mode = fine_sweep_cached_plan<T>(f.N, nrhs, p, maxcnt, &q);
  if (mode == 0 || (mode != 1 && fz.any())) return false;
  if (mode == 3) {
    hipLaunchKernelGGL((k_kaczmarz_fine_pipe<T>), dim3((unsigned)(q.ntu * q.ntv), (unsigned)nrhs), dim3(FP_NT), 0, s,
                       f, q, xin, xout, b);
    return true;
  }
  const dim3 grid((unsigned)(p.ntu * p.ntv), (unsigned)nrhs);
  if (mode == 2) {
    constexpr int UB = 36 * (int)sizeof(cx<T>) / 16, US = 2 * (int)sizeof(cx<T>) / 16;
    const bool it2 = maxcnt <= 2 * FSS_GROUPS, sb4 = maxcnt * (UB + 2 * US) <= 4 * FSS_NT;
#define FSS_LAUNCH(I, S)                                                                                          \
  hipLaunchKernelGGL((k_kaczmarz_fine_sweep_s<T, FS_LDS_LARGE, I, S>), grid, dim3(FSS_NT), 0, s, f, p, maxcnt, xin, \
                     xout, b)
    constexpr int SBM = FSS_SB_MAX<T>;
    if (it2 && sb4) FSS_LAUNCH(2, 4);
    else if (it2) FSS_LAUNCH(2, SBM);
    else if (sb4) FSS_LAUNCH(4, 4);
    else FSS_LAUNCH(4, SBM);  // (SBM = 4 for FP64: the plan keeps its colours within 4 loads per thread)
#undef FSS_LAUNCH
    return true;
  }
  const size_t lds = fine_sweep_lds<T>(p);
  maxcnt = 0;
  for (int c = 0; c < 16; ++c) maxcnt = std::max(maxcnt, p.first[c + 1] - p.first[c]);
#define FS_LAUNCH(L, I) \
  hipLaunchKernelGGL((k_kaczmarz_fine_sweep<T, L, I>), grid, dim3(FS_NT), 0, s, f, p, xin, xout, b, fz)
#define FS_ITER(L)                     \
  do {                                 \
    if (maxcnt <= FS_GROUPS)           \
      FS_LAUNCH(L, 1);                 \
    else                               \
      FS_LAUNCH(L, 2);                 \
  } while (0)
  if (lds <= (size_t)FS_LDS_TINY)
    FS_ITER(FS_LDS_TINY);
  else if (lds <= (size_t)FS_LDS_SMALL)
    FS_ITER(FS_LDS_SMALL);
  else
    FS_ITER(FS_LDS_LARGE);
#undef FS_ITER
#undef FS_LAUNCH
  return true;
}
// The plan of form (0: the library's choice, 1, 2, 3) for the plan query of
// the C ABI; returns the form written, 0 for none.  sched = {A, M, W} of the
// pipelined form, zeros for the others.
int fine_sweep_plan_query(int N, int nrhs, bool fp32, int form, FineSweepPlan& p, int sched[3]) {
  int maxcnt = 0;
  sched[0] = sched[1] = sched[2] = 0;
  FinePipePlan q;
  int got = 0;
  if (form == 3) got = fine_pipe_choose(N, nrhs, q, p) ? 3 : 0;
  else if (form == 0)
    got = fp32 ? fine_sweep_cached_plan<float>(N, nrhs, p, maxcnt, &q)
               : fine_sweep_cached_plan<double>(N, nrhs, p, maxcnt, &q);
  if (got == 3) {
    sched[0] = q.A;
    sched[1] = q.M;
    sched[2] = FP_W;
  }
  if (form == 0 || form == 3) return got;
  if (form == 1) return (fp32 ? fine_sweep_choose<float>(N, nrhs, p) : fine_sweep_choose<double>(N, nrhs, p)) ? 1 : 0;
  return (fp32 ? fine_sweep_choose_s<float>(N, nrhs, p, maxcnt) : fine_sweep_choose_s<double>(N, nrhs, p, maxcnt)) ? 2 : 0;
}

template bool fine_sweep_applies<double>(const FineT<double>&, int);
template bool fine_sweep_applies<float>(const FineT<float>&, int);
template bool fine_sweep_fusable<double>(const FineT<double>&, int);
template bool fine_sweep_fusable<float>(const FineT<float>&, int);
template bool launch_fine_sweep<double>(const FineT<double>&, const zd*, zd*, const zd*, int, hipStream_t,
                                        const FineFuse<double>&);
template bool launch_fine_sweep<float>(const FineT<float>&, const zf*, zf*, const zf*, int, hipStream_t,
                                       const FineFuse<float>&);

template void launch_smooth_fine_il<double>(const FineT<double>&, int, int, zd*, const zd*, zd*, zd*, int, int,
                                            hipStream_t);
template void launch_smooth_fine_il<float>(const FineT<float>&, int, int, zf*, const zf*, zf*, zf*, int, int,
                                           hipStream_t);

template void launch_kaczmarz_fine<double>(const FineT<double>&, int, int, zd*, const zd*, int, hipStream_t,
                                           const double*);
template void launch_kaczmarz_fine<float>(const FineT<float>&, int, int, zf*, const zf*, int, hipStream_t,
                                          const double*);

// ---------------------------------------------------------------------------
// Transfers between level 0 and the 4x4 aggregates of the half-x grid.
// Aggregate a = Ay*(NH/4) + Ax holds the even sites xh = 4Ax + lx, y = 4Ay + ly,
// local row 4*ly + lx.  rc[a][8s + k] = sum_row conj(P[a][s][row][k]) r[site][s].
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_restrict_fine(FineT<T> f, const cx<T>* __restrict__ P, const cx<T>* __restrict__ r, cx<T>* __restrict__ rc,
                                cx<T>* __restrict__ xz) {
  using C = cx<T>;
  const int cxn = f.NH / 4, cyn = f.N / 4;
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cxn * cyn * 16) return;
  const int a = t >> 4, d = t & 15, s = d >> 3, k = d & 7;
  const int Ax = a % cxn, Ay = a / cxn;
  const size_t n = (size_t)f.N * f.NH * 2, nc = (size_t)cxn * cyn * 16;
  const C* rv = r + blockIdx.y * n;
  const C* Pa = P + ((size_t)a * 2 + s) * 16 * 8;
  C acc = {0, 0};
  for (int row = 0; row < 16; ++row) {
    int ly = row >> 2, lx = row & 3;
    int e = (4 * Ay + ly) * f.NH + 4 * Ax + lx;
    acc = acc + cjmul_fixed(Pa[row * 8 + k], rv[2 * e + s]);
  }
  rc[blockIdx.y * nc + t] = acc;
  if (xz) xz[blockIdx.y * nc + t] = C{0, 0};  // the coarse level's zero initial guess
}

template <typename T>
void launch_restrict_fine(const FineT<T>& f, const cx<T>* P, const cx<T>* r, cx<T>* rc, int nrhs, hipStream_t s,
                          cx<T>* xz) {
  int n = (f.NH / 4) * (f.N / 4) * 16;
  hipLaunchKernelGGL(k_restrict_fine<T>, dim3((n + 255) / 256, nrhs), dim3(256), 0, s, f, P, r, rc, xz);
}

template <typename T>
__global__ void k_prolong_fine(FineT<T> f, const cx<T>* __restrict__ P, const cx<T>* __restrict__ xc, cx<T>* __restrict__ x) {
  const int cxn = f.NH / 4, cyn = f.N / 4;
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= f.N * f.NH * 2) return;
  const int e = t >> 1, s = t & 1;
  const size_t n = (size_t)f.N * f.NH * 2, nc = (size_t)cxn * cyn * 16;
  x[blockIdx.y * n + t] = x[blockIdx.y * n + t] + fine_prolong_entry(f, P, xc + blockIdx.y * nc, e, s);
}

template <typename T>
void launch_prolong_fine(const FineT<T>& f, const cx<T>* P, const cx<T>* xc, cx<T>* x, int nrhs, hipStream_t s) {
  int n = f.N * f.NH * 2;
  hipLaunchKernelGGL(k_prolong_fine<T>, dim3((n + 255) / 256, nrhs), dim3(256), 0, s, f, P, xc, x);
}
template void launch_restrict_fine<double>(const FineT<double>&, const zd*, const zd*, zd*, int, hipStream_t,
                                           zd*);
template void launch_restrict_fine<float>(const FineT<float>&, const zf*, const zf*, zf*, int, hipStream_t,
                                           zf*);
template void launch_prolong_fine<double>(const FineT<double>&, const zd*, const zd*, zd*, int, hipStream_t);
template void launch_prolong_fine<float>(const FineT<float>&, const zf*, const zf*, zf*, int, hipStream_t);

// ---------------------------------------------------------------------------
// Galerkin product D_1 = P^H Dhat P, assembled per aggregate A by fine
// displacement: for every fine pair (i in A, j = i + disp) the aggregate of j
// (in unwrapped coordinates) fixes the offset o, so grids of extent < 3 (where
// offsets alias) are still exact.
// D_1[A][o][(s1,k1),(s2,k2)] = sum conj(P_A[s1][i][k1]) Dhat[(i,s1),(j,s2)] P_{A+o}[s2][j][k2]
// ---------------------------------------------------------------------------
__device__ __forceinline__ int offset_index(int dx, int dy) {
  if (dx == 0 && dy == 0) return 0;
  if (dx == 1 && dy == 0) return 1;
  if (dx == -1 && dy == 0) return 2;
  if (dx == 0 && dy == 1) return 3;
  if (dx == 0 && dy == -1) return 4;
  if (dx == 1 && dy == 1) return 5;
  if (dx == -1 && dy == -1) return 6;
  return -1;
}

__device__ __forceinline__ int floordiv(int a, int b) { return (a >= 0) ? a / b : -((-a + b - 1) / b); }

__global__ __launch_bounds__(256) void k_galerkin_fine(Fine f, const zd* __restrict__ P, zd* __restrict__ D1) {
  const int cxn = f.NH / 4, cyn = f.N / 4;
  const int A = blockIdx.x, Ax = A % cxn, Ay = A / cxn;
  __shared__ zd rows[16][9][2][2];
  __shared__ int tgt_o[16][9], tgt_row[16][9], tgt_agg[16][9];
  const int tid = threadIdx.x;
  if (tid < 16) {
    const int ly = tid >> 2, lx = tid & 3;
    const int y = 4 * Ay + ly, xh = 4 * Ax + lx;
    zd e[9][2][2];
    int jn[9];
    dhat_rows(f, xh, y, e, jn);
    const int x = 2 * xh + (y & 1);
    for (int q = 0; q < 9; ++q) {
      for (int s = 0; s < 2; ++s)
        for (int t = 0; t < 2; ++t) rows[tid][q][s][t] = e[q][s][t];
      // unwrapped half-x coordinates of the neighbour
      const int yn = y + SDY[q];
      const int xn = x + SDX[q];
      const int xhn = (xn >= 0) ? (xn >> 1) : -((-xn + 1) >> 1);
      const int Axn = floordiv(xhn, 4), Ayn = floordiv(yn, 4);
      tgt_o[tid][q] = offset_index(Axn - Ax, Ayn - Ay);
      tgt_row[tid][q] = 4 * (yn - 4 * Ayn) + (xhn - 4 * Axn);
      tgt_agg[tid][q] = wrapn(Ayn, cyn) * cxn + wrapn(Axn, cxn);
    }
  }
  __syncthreads();
  for (int out = tid; out < NOFF * 256; out += blockDim.x) {
    const int o = out >> 8, rr = (out >> 4) & 15, cc = out & 15;
    const int s1 = rr >> 3, k1 = rr & 7, s2 = cc >> 3, k2 = cc & 7;
    zd acc = {0, 0};
    for (int i = 0; i < 16; ++i) {
      const zd pa = P[(((size_t)A * 2 + s1) * 16 + i) * 8 + k1];
      zd part = {0, 0};
      for (int q = 0; q < 9; ++q) {
        if (tgt_o[i][q] != o) continue;
        const zd pb = P[(((size_t)tgt_agg[i][q] * 2 + s2) * 16 + tgt_row[i][q]) * 8 + k2];
        part = part + rows[i][q][s1][s2] * pb;
      }
      acc = acc + cjmul(pa, part);
    }
    D1[(((size_t)A * NOFF + o) * 16 + rr) * 16 + cc] = acc;
  }
}

void launch_galerkin_fine(const Fine& f, const zd* P, zd* D1, hipStream_t s) {
  int na = (f.NH / 4) * (f.N / 4);
  hipLaunchKernelGGL(k_galerkin_fine, dim3(na), dim3(256), 0, s, f, P, D1);
}

// ---------------------------------------------------------------------------
// Least-squares fit (Sec. 3.3, eq. LSfuncrowi) per aggregate and spin: with
// k <= 8 test vectors restricted to a block of R rows the fit is exact and
// P_{a,s} is the orthonormal basis from classical Gram-Schmidt applied twice
// (positive R_jj), in test-vector order.  R rows of one problem live in R
// consecutive lanes; sums are butterfly reductions over those lanes.
// ---------------------------------------------------------------------------
template <int R>
__device__ __forceinline__ zd seg_sum(zd v) {
#pragma unroll
  for (int off = R / 2; off > 0; off >>= 1) {
    v.x += __shfl_xor(v.x, off, 64);
    v.y += __shfl_xor(v.y, off, 64);
  }
  return v;
}

template <int R>
__device__ void cgs2_fit(const zd* vrow, int k, zd* qrow) {
  // vrow[j]: the lane's entry of test vector j; qrow[j]: output
  for (int j = 0; j < 8; ++j) qrow[j] = zd{0, 0};
  for (int j = 0; j < k && j < 8; ++j) {
    zd w = vrow[j];
    for (int pass = 0; pass < 2; ++pass) {
      zd h[8];
      for (int q = 0; q < j; ++q) h[q] = seg_sum<R>(cjmul(qrow[q], w));
      for (int q = 0; q < j; ++q) w = w - qrow[q] * h[q];
    }
    const double nrm = sqrt(seg_sum<R>(zd{norm2(w), 0.0}).x);
    qrow[j] = nrm > 0 ? cdiv_real(w, nrm) : zd{0, 0};
  }
}

__global__ __launch_bounds__(64) void k_fit_fine(Fine f, const zd* __restrict__ V, int k, zd* __restrict__ P) {
  const int cxn = f.NH / 4, cyn = f.N / 4;
  const int lane = threadIdx.x, grp = lane >> 4, row = lane & 15;
  const int prob = blockIdx.x * 4 + grp;  // (aggregate, spin)
  const int nprob = cxn * cyn * 2;
  const bool act = prob < nprob;
  const int a = act ? prob >> 1 : 0, s = prob & 1;
  const int Ax = a % cxn, Ay = a / cxn;
  const int e = (4 * Ay + (row >> 2)) * f.NH + 4 * Ax + (row & 3);
  const size_t n = (size_t)f.N * f.NH * 2;
  zd v[8], q[8];
  for (int j = 0; j < 8; ++j) v[j] = (act && j < k) ? V[j * n + 2 * e + s] : zd{0, 0};
  cgs2_fit<16>(v, k, q);
  if (act)
    for (int j = 0; j < 8; ++j) P[(((size_t)a * 2 + s) * 16 + row) * 8 + j] = q[j];
}

void launch_fit_fine(const Fine& f, const zd* V, int k, zd* P, hipStream_t s) {
  int nprob = (f.NH / 4) * (f.N / 4) * 2;
  hipLaunchKernelGGL(k_fit_fine, dim3((nprob + 3) / 4), dim3(64), 0, s, f, V, k, P);
}

// ---------------------------------------------------------------------------
// Test vectors: Philox4x32-10 (Salmon et al., SC'11) keyed by the seed with
// counter (dof, vector, 0, 0); two 53-bit uniforms in (0,1) -> Box-Muller ->
// one complex Gaussian with Re, Im i.i.d. N(0, 1/2).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
    const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
  }
}

__global__ void k_philox_tv(int n, int k, uint64_t seed, zd* __restrict__ out) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (size_t)n * k) return;
  const int j = (int)(t / n), d = (int)(t - (size_t)j * n);
  uint32_t c[4] = {(uint32_t)d, (uint32_t)j, 0u, 0u};
  philox10(c, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
  const double two53 = 9007199254740992.0;
  const double u1 = ((double)(c[0] >> 5) * 67108864.0 + (double)(c[1] >> 6) + 0.5) / two53;
  const double u2 = ((double)(c[2] >> 5) * 67108864.0 + (double)(c[3] >> 6) + 0.5) / two53;
  const double rho = sqrt(-2.0 * log(u1));
  const double th = 2.0 * M_PI * u2;
  const double s2 = sqrt(2.0);
  out[t] = zd{rho * cos(th) / s2, rho * sin(th) / s2};
}

void launch_philox_tv(int n, int k, uint64_t seed, zd* out, hipStream_t s) {
  size_t tot = (size_t)n * k;
  hipLaunchKernelGGL(k_philox_tv, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, k, seed, out);
}

}  // namespace bamg
