// Internal declarations of libbamg: complex arithmetic, device data layouts of
// the levels and the host-side launch wrappers of every kernel.
//
// Device layouts (all FP64 unless a template says otherwise):
//   links   Ue[(y*NH + xh)*2 + mu], Uo likewise: the two forward links of the
//           even / odd site with half-x index (xh, y); NH = N/2.  The half-x
//           index of lattice site (x, y) is y*NH + (x >> 1) for both parities.
//   level 0 vectors v[rhs][y*NH + xh][s]   (the reduced layout of the ABI)
//   level l vectors v[rhs][site][16]       (dof 8 s + k)
//   P_l     [agg][s][row][8]
//   D_l     [site][7][16][16]   offsets (0,0) (+1,0) (-1,0) (0,+1) (0,-1) (+1,+1) (-1,-1)
//   Kinv_l  [site][16][16]      inverse of the lower triangle of G = A_a A_a^H
//                               (the block row A_a of site a), used to run the
//                               16 sequential row projections of a site at once
#pragma once
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace bamg {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T x, y;
};
using zd = cx<double>;
using zf = cx<float>;
// reduced-precision storage of complex operator entries (accumulated in FP32)
struct alignas(4) hcx {
  __half x, y;
};
struct alignas(4) bcx {
  __hip_bfloat16 x, y;
};
template <typename T>
__device__ __forceinline__ cx<T> widen(cx<double> v) { return {(T)v.x, (T)v.y}; }
template <typename T>
__device__ __forceinline__ cx<T> widen(cx<float> v) { return {(T)v.x, (T)v.y}; }
template <typename T>
__device__ __forceinline__ cx<T> widen(hcx v) { return {(T)__half2float(v.x), (T)__half2float(v.y)}; }
template <typename T>
__device__ __forceinline__ cx<T> widen(bcx v) { return {(T)__bfloat162float(v.x), (T)__bfloat162float(v.y)}; }

template <typename T>
__host__ __device__ __forceinline__ cx<T> cmk(T a, T b) { return cx<T>{a, b}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a) { return {-a.x, -a.y}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return {s * a.x, s * a.y}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> conj(cx<T> a) { return {a.x, -a.y}; }
// conj(a) * b
template <typename T>
__host__ __device__ __forceinline__ cx<T> cjmul(cx<T> a, cx<T> b) {
  return {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}
// i * a
template <typename T>
__host__ __device__ __forceinline__ cx<T> mul_i(cx<T> a) { return {-a.y, a.x}; }
template <typename T>
__host__ __device__ __forceinline__ T norm2(cx<T> a) { return a.x * a.x + a.y * a.y; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> cdiv_real(cx<T> a, T s) { return {a.x / s, a.y / s}; }

// Complex product with its contraction fixed: each component is one fused
// multiply-add on the exactly rounded other product, whatever the compiler
// would otherwise fuse, so every kernel that evaluates the same product gets
// the same bits (kernels chosen by problem size must agree).
template <typename T>
__device__ __forceinline__ cx<T> cmul_fixed(cx<T> a, cx<T> b) {
  return cx<T>{fma(a.x, b.x, -(a.y * b.y)), fma(a.x, b.y, a.y * b.x)};
}
// conj(a) b with its contraction fixed
template <typename T>
__device__ __forceinline__ cx<T> cjmul_fixed(cx<T> a, cx<T> b) {
  return cx<T>{fma(a.x, b.x, a.y * b.y), fma(a.x, b.y, -(a.y * b.x))};
}

// Work-group p of a launch goes to XCD p mod 8 (the chip's 8 XCDs, each with
// its own L2, take work-groups in turn).  xcd_block renumbers the nb
// work-groups so that each XCD takes one contiguous range, in order: logical
// neighbours run on one XCD at about the same time and share its L2.
__device__ __forceinline__ unsigned xcd_block(unsigned p, unsigned nb) {
  const unsigned k = p & 7, q = nb >> 3, rem = nb & 7;
  return k * q + (k < rem ? k : rem) + (p >> 3);
}

// Lane exchange by DPP moves (within rows of 16 lanes; no LDS round trip).
// CTRL: quad permutations (0x00-0xFF), row shifts left / right by n (0x100 + n /
// 0x110 + n: lane i reads lane i + n / i - n of its row), row rotations right
// by n (0x120 + n).  A lane whose source lies outside the row reads 0.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
constexpr int DPP_QUAD_XOR1 = 0xB1, DPP_QUAD_XOR2 = 0x4E;  // quad_perm [1,0,3,2] and [2,3,0,1]
constexpr int DPP_ROW_SHL4 = 0x104, DPP_ROW_SHR4 = 0x114, DPP_ROW_ROR4 = 0x124, DPP_ROW_ROR8 = 0x128;

constexpr int NOFF = 7;  // coarse stencil offsets
constexpr int NC = 16;   // dofs per coarse site

// Fine-level geometry and links (links in the arithmetic type T)
template <typename T>
struct FineT {
  int N = 0, NH = 0;
  double c = 0, kappa = 0, kappa2 = 0;  // c = m + 2, kappa = 1/c
  const cx<T>* Ue = nullptr;
  const cx<T>* Uo = nullptr;
  const cx<T>* Bst = nullptr;  // stored slot blocks of Dhat, [site][9][4] (smoother)
  const cx<T>* Gst = nullptr;  // per even site (nu_0, nu_1), G_10 of its row pair (smoother)
};
using Fine = FineT<double>;

// ---- fine.hip ---------------------------------------------------------------
void launch_gauge_pack(const zd* U, zd* Ue, zd* Uo, int N, hipStream_t s);
void launch_eo_reduce(const Fine& f, const zd* b, zd* bh, int nrhs, hipStream_t s);
void launch_eo_reconstruct(const Fine& f, const zd* b, const zd* xe, zd* x, int nrhs, hipStream_t s);
// y = Dhat x, or y = b - Dhat x if b != nullptr  (T = double or float)
template <typename T>
void launch_dhat(const FineT<T>& f, const cx<T>* x, cx<T>* y, const cx<T>* b, int nrhs, hipStream_t s);
// Bst[site][slot][4]: the 2x2 blocks of Dhat coupling each even site to its 9
// stencil slots (built from the links)
template <typename T>
void launch_slot_blocks(const FineT<T>& f, cx<T>* Bst, hipStream_t s);
// Gst[site] = ((nu_0, nu_1), G_10): the squared row norms and the Gram entry
// of the site's row pair, from Bst, with the smoother's own expressions and
// lane sums (the same bits as forming them in a pass)
template <typename T>
void launch_slot_gram(const FineT<T>& f, const cx<T>* Bst, cx<T>* Gst, hipStream_t s);
// one colour pass over the nsites = N^2/32 sites of fine colour `colour`
// (lam != NULL: per right-hand side shift lam[r], the pass on (Dhat - lam Gamma_5) x = 0)
template <typename T>
void launch_kaczmarz_fine(const FineT<T>& f, int colour, int nsites, cx<T>* x, const cx<T>* b, int nrhs,
                          hipStream_t s, const double* lam = nullptr);
// count fine sweeps for R >= 16 right-hand sides through the right-hand-side
// interleaved layout (xi, bi: n R entries each; b may be NULL for b = 0);
// bitwise the same as count sweeps of launch_kaczmarz_fine
template <typename T>
void launch_smooth_fine_il(const FineT<T>& f, int ncol, int per_colour, cx<T>* x, const cx<T>* b, cx<T>* xi,
                           cx<T>* bi, int R, int count, hipStream_t s);
// One fine sweep (the 16 colour passes) per launch, blocked in LDS: xout is
// bitwise what the 16 launches of launch_kaczmarz_fine make of xin.  xin and
// xout must not overlap.  fine_sweep_applies is false where no tile plan
// applies (small lattices, no stored slot blocks); the caller then runs the
// colour passes.
struct FineSweepPlan {
  int Tu, Tv, ntu, ntv;      // tile extents in (u, v) and tile counts
  int i0, j0, Ru, Rv;        // region origin relative to the tile origin, region extents
  int nupd;                  // projections per tile
  int first[17];             // first projection of colour c
  int si0[16], sj0[16], nj[16];  // colour c: first site (relative to the tile origin), sites along v
};
template <typename T>
bool fine_sweep_applies(const FineT<T>& f, int nrhs);
// the plan of form 0 (the library's choice), 1 (LDS-resident) or 2
// (streaming); returns the form written, 0 for none (host only)
int fine_sweep_plan_query(int N, int nrhs, bool fp32, int form, FineSweepPlan& p, int sched[3]);
// Work a sweep of the LDS-resident form can take over from the launches
// around it (all fields optional):
// - P, xc: every x value the sweep reads is x + P xc, the prolongation of
//   launch_prolong_fine with the same bits (xin itself is not changed);
// - xzero: x is taken as zero and xin is not read;
// - b64, b_out: b is read as b64 (FP64) rounded to T, and written rounded to
//   b_out on the work-group's tile (b is not read; b_out may be b);
// - x64: the result is written in FP64 to x64 instead of to xout.
template <typename T>
struct FineFuse {
  const cx<T>* P = nullptr;
  const cx<T>* xc = nullptr;
  bool xzero = false;
  const zd* b64 = nullptr;
  cx<T>* b_out = nullptr;
  zd* x64 = nullptr;
  bool any() const { return P || xzero || b64 || x64; }
};
// true where launch_fine_sweep takes the LDS-resident form, the one that
// carries FineFuse work
template <typename T>
bool fine_sweep_fusable(const FineT<T>& f, int nrhs);
// false (nothing launched) if fz asks for work and the size takes another form
template <typename T>
bool launch_fine_sweep(const FineT<T>& f, const cx<T>* xin, cx<T>* xout, const cx<T>* b, int nrhs, hipStream_t s,
                       const FineFuse<T>& fz = FineFuse<T>{});
// rc = P^H r (level 0 -> 1), and xz = 0 (level 1, same layout) if xz != NULL;
// x += P xc (level 1 -> 0)
template <typename T>
void launch_restrict_fine(const FineT<T>& f, const cx<T>* P, const cx<T>* r, cx<T>* rc, int nrhs, hipStream_t s,
                          cx<T>* xz = nullptr);
template <typename T>
void launch_prolong_fine(const FineT<T>& f, const cx<T>* P, const cx<T>* xc, cx<T>* x, int nrhs, hipStream_t s);
// rc = P^H (b - Dhat x) in one launch, the bits of launch_dhat then
// launch_restrict_fine (r itself is not stored), and xz = 0 if not null;
// false (nothing launched) where the lattice does not take its tiles
template <typename T>
bool launch_residual_restrict_fine(const FineT<T>& f, const cx<T>* P, const cx<T>* x, const cx<T>* b, cx<T>* rc,
                                   int nrhs, hipStream_t s, cx<T>* xz = nullptr);
// D_1 = P^H Dhat P in 7-offset blocks
void launch_galerkin_fine(const Fine& f, const zd* P, zd* D1, hipStream_t s);
// gather test vectors into aggregate blocks and fit P (level 0)
void launch_fit_fine(const Fine& f, const zd* V, int k, zd* P, hipStream_t s);
void launch_philox_tv(int n, int k, uint64_t seed, zd* out, hipStream_t s);

// ---- coarse.hip -------------------------------------------------------------
// coarse level: arithmetic type T, operator storage type S (cx<double>,
// cx<float>, hcx or bcx); Kinv in T
template <typename T, typename S>
struct CoarseT {
  int ex = 0, ey = 0;  // extents in sites
  const S* D = nullptr;
  const cx<T>* Kinv = nullptr;
};
using Coarse = CoarseT<double, zd>;
template <typename T, typename S>
void launch_coarse_apply(const CoarseT<T, S>& c, const cx<T>* x, cx<T>* y, const cx<T>* b, int nrhs, hipStream_t s);
// one colour pass; mode 8 / 16: the 8- or 16-colouring, mode 1: one site per colour
template <typename T, typename S>
void launch_kaczmarz_coarse(const CoarseT<T, S>& c, int colour, int mode, int nsites, cx<T>* x, const cx<T>* b,
                            int nrhs, hipStream_t s);
// colours c and c + 1 (c even) of the 8-colouring in one launch, out of place
// (xin and xout must not overlap), bitwise the two colour passes; where
// coarse_pair_applies.  With xc != NULL the launch starts from xin + P xc
// (P: the level's interpolation from the next level, xc: that level's x),
// bitwise a prolongation followed by the two passes.
bool coarse_pair_applies(int ex, int ey, int mode);
template <typename T, typename S>
void launch_kaczmarz_coarse_pair(const CoarseT<T, S>& c, int colour, int nsites, const cx<T>* xin, cx<T>* xout,
                                 const cx<T>* b, int nrhs, hipStream_t s, const cx<T>* P = nullptr,
                                 const cx<T>* xc = nullptr);
// y = D x or b - D x on the matrix cores (FP32 arithmetic, 16 RHS per work-group)
template <typename S>
void launch_coarse_apply_mfma(const CoarseT<float, S>& c, const zf* x, zf* y, const zf* b, int nrhs, hipStream_t s);
// the same pass on the matrix cores (FP32 arithmetic, one wave per site and 16 RHS)
template <typename S>
void launch_kaczmarz_coarse_mfma(const CoarseT<float, S>& c, int colour, int mode, int nsites, zf* x, const zf* b,
                                 int nrhs, hipStream_t s);
// Kinv (type T) from the stored operator (type S), computed in FP64
template <typename T, typename S>
void launch_kaczmarz_prep(const CoarseT<T, S>& c, cx<T>* Kinv, hipStream_t s);
// level l (ex x ey) -> l+1 (ex/2 x ey/2); xz as for launch_restrict_fine
template <typename T>
void launch_restrict_coarse(int ex, int ey, const cx<T>* P, const cx<T>* r, cx<T>* rc, int nrhs, hipStream_t s,
                            cx<T>* xz = nullptr);
template <typename T>
void launch_prolong_coarse(int ex, int ey, const cx<T>* P, const cx<T>* xc, cx<T>* x, int nrhs, hipStream_t s);
// rc = P^H (b - D x) from level l (c, ex x ey) to l+1 in one launch, xz as
// for launch_restrict_coarse: the same bits as launch_coarse_apply followed by
// launch_restrict_coarse; false (nothing launched) without b or for odd extents
template <typename T, typename S>
bool launch_residual_restrict_coarse(const CoarseT<T, S>& c, const cx<T>* P, const cx<T>* x, const cx<T>* b,
                                     cx<T>* rc, int nrhs, hipStream_t s, cx<T>* xz = nullptr);
void launch_galerkin_coarse(const Coarse& c, const zd* P, zd* Dc, hipStream_t s);
void launch_fit_coarse(const Coarse& c, const zd* V, int k, zd* P, hipStream_t s);
// expand the block stencil into a dense n x n matrix (coarsest level)
void launch_densify(const Coarse& c, zd* A, hipStream_t s);

// ---- dense.hip --------------------------------------------------------------
// In-place Gauss-Jordan inversion with partial pivoting of the n x n matrix A;
// in-place inverse of the n x n row-major A by blocked Gauss-Jordan elimination
// with partial pivoting (row interchanges recorded in perm[n]); T holds
// gj_workspace(n) complex; sets *flag = 1 on a zero pivot.  The inverse's
// columns are put back in order by launch_gj_unpermute.
size_t gj_workspace(int n);
void launch_gj_invert(zd* A, int n, zd* T, int* perm, int* flag, hipStream_t s);
void launch_gj_unpermute(zd* A, int n, const int* perm, hipStream_t s);
// y = A x for nrhs vectors (A n x n row-major): one wave per row for few
// right-hand sides, an LDS-tiled product (A read once per 32 RHS) for many
// (or whenever `many` is set; work holds dense_mm_workspace(n, nrhs) complex)
void launch_dense_mv(const zd* A, int n, const zd* x, zd* y, int nrhs, bool many, zd* work, hipStream_t s);
// the same product with the FP64 inverse for complex64 x and y (x widened
// exactly, sums in FP64, y rounded to nearest): bitwise the conversions
// around launch_dense_mv, in one launch where it takes one wave per row
// (returns false, launching nothing, otherwise)
bool launch_dense_mv_f32io(const zd* A, int n, const zf* x, zf* y, int nrhs, bool many, hipStream_t s);
// The single-RHS coarsest product from the 64 x 64 blocks on and above the
// block diagonal of the gamma5-Hermitian inverse (n % 64 == 0).  blk: the
// (I, J) pairs of the packed blocks, I <= J, row by row; part: 2 (n / 64)^2 * 64
// entries.  The product returns false (and launches nothing) unless Ap is set
// and nrhs is 1 or 2.
void launch_pack_g5(const zd* A, int n, const int* blk, zd* Ap, hipStream_t s);
bool launch_dense_mv_g5(const zd* Ap, const int* blk, int n, const zd* x, zd* y, int nrhs, zd* part, hipStream_t s);
bool launch_dense_mv_g5_f32io(const zd* Ap, const int* blk, int n, const zf* x, zf* y, int nrhs, zd* part,
                              hipStream_t s);
// the same from an FP32 copy of the packed blocks (rounded to nearest from the
// averaged FP64 blocks), products and sums in FP64 (the mixed cycle with
// coarsest_fp32)
void launch_pack_g5_f32(const zd* A, int n, const int* blk, zf* Ap, hipStream_t s);
bool launch_dense_mv_g5_c32(const zf* Ap, const int* blk, int n, const zf* x, zf* y, int nrhs, zd* part,
                            hipStream_t s);
size_t dense_mm_workspace(int n, int nrhs);
// FP32 operands (mixed-precision cycle): y = A x with A the n x n FP32 copy of
// the coarsest inverse, n a multiple of 16; one wave per row for up to two
// right-hand sides, else split-K MFMA tiles with
// dense_mm32_workspace_bytes(n, nrhs) bytes of partials in work
void launch_dense_mv32(const zf* A, int n, const zf* x, zf* y, int nrhs, bool many, zf* work, hipStream_t s);
size_t dense_mm32_workspace_bytes(int n, int nrhs);

// ---- blas.hip ---------------------------------------------------------------
// partial[b][v] = sum over block b of conj(X_v) w, X_v = X + v*ldx; then out[v] = sum_b partial[b][v]
int blas_nblocks(size_t n);
// the finer blocks of the batched forms below and of launch_norms with fine =
// true (the FGMRES of bamg_solve / fgmres_batch, whose launches hold few
// vectors): 512 entries each, at most 512 blocks; never fewer than
// blas_nblocks(n), at most 4 times as many
int blas_nblocks_fine(size_t n);
void launch_multidot(const zd* X, size_t ldx, int nv, const zd* w, size_t n, zd* partial, zd* out,
                     hipStream_t s);
// w += sign * sum_v X_v h_v   (h on device)
void launch_multiaxpy(const zd* X, size_t ldx, int nv, const zd* h, double sign, zd* w, size_t n,
                      hipStream_t s);
// per-vector squared norms of nv vectors of length n: out[v] (real part);
// vector v at X + map[v] * ldx when map (device) is given, else X + v * ldx
void launch_norms(const zd* X, size_t ldx, int nv, size_t n, zd* partial, zd* out, hipStream_t s,
                  const int* map = nullptr, bool fine = false);
// X_v *= 1/sqrt(nrm[v].x) for nrm > 0
void launch_normalize(zd* X, size_t ldx, int nv, size_t n, const zd* nrm, hipStream_t s);
// y = alpha x (alpha real, host scalar)
void launch_scale_copy(const zd* x, zd* y, size_t n, double alpha, hipStream_t s);
void launch_fill_zero(zd* x, size_t n, hipStream_t s);
// x -= z
void launch_sub(const zd* z, zd* x, size_t n, hipStream_t s);
// zero `bytes` bytes (a multiple of 8) with a kernel (no memset node)
void launch_zero(void* p, size_t bytes, hipStream_t s);
void launch_copy(const zd* x, zd* y, size_t n, hipStream_t s);
// flag[0] = 1 if any entry of x is not finite
void launch_check_finite(const zd* x, size_t n, int* flag, hipStream_t s);
// element-wise precision conversion (complex): out[i] = in[i] rounded to the
// output type (round to nearest)
template <typename Tin, typename Tout>
void launch_convert(const Tin* in, Tout* out, size_t n, hipStream_t s);
// out = in rounded to FP32, zero_out = 0 (n entries each)
void launch_convert_zero(const zd* in, zf* out, zf* zero_out, size_t n, hipStream_t s);
// batched forms over R right-hand sides: basis vector v of right-hand side r
// at X + (v*R + r)*n, w_r at W + r*n, coefficients at stride 64 per r
// (host_out, if not null: pinned host memory laid out as out that receives a
// copy of the results from the reduction kernel itself)
void launch_bmultidot(const zd* X, int nv, const zd* W, size_t n, int R, zd* partial, zd* out, hipStream_t s,
                      zd* host_out = nullptr);
void launch_bmultiaxpy(const zd* X, int nv, const zd* h, double sign, zd* W, size_t n, int R, hipStream_t s);
// W_r += sign sum_{v < nv} X_{v,r} h[r][v], then out[r][v] = X_{v,r}^H W_r for
// v < nd (nd > 0) or out[r] = |W_r|^2 (nd = 0), in one pass over W_r per
// launch pair (nd = 0 and out null: only the block partials of |W_r|^2, for
// launch_norm_scale); false (nothing launched) where a chunk is too long
bool launch_baxpy_dot(const zd* X, int nv, const zd* h, double sign, zd* W, size_t n, int R, int nd, zd* partial,
                      zd* out, hipStream_t s, zd* host_out = nullptr);
bool baxpy_dot_applies(size_t n);
// y_r = c[r] x_r (c device, real)
void launch_bscale(const zd* x, zd* y, size_t n, int R, const double* c, hipStream_t s);
// one vector: y = x / sqrt(nrm2[0].x)
void launch_bscale_rnorm(const zd* x, zd* y, size_t n, const zd* nrm2, hipStream_t s);
// one vector: out[0] (and host_out) = |w|^2 from the block partials that
// launch_baxpy_dot with nd = 0 and out = nullptr leaves, and y = w / |w|, in
// one launch (the bits of the reduction and launch_bscale_rnorm)
void launch_norm_scale(const zd* partial, const zd* w, zd* y, size_t n, zd* out, zd* host_out, hipStream_t s);
// x_r += sum_q Z_{q,r} y[r*64 + q]
void launch_blincomb(const zd* Z, int nq, const zd* y, zd* x, size_t n, int R, hipStream_t s);
// slot-mapped forms (continuous batching): entry a of a launch uses slot slot[a]
// (device int arrays); vector v of that slot at X + slot[a]*lds + v*ldv, the
// first cnt[a] vectors; gathered vectors contiguous at W + a*n; coefficients
// at stride 64 per entry.  Per entry the arithmetic equals the batched forms.
void launch_smultidot(const zd* X, size_t lds, size_t ldv, const int* slot, const int* cnt, int maxcnt, const zd* W,
                      size_t n, int A, zd* partial, zd* out, hipStream_t s);
void launch_smultiaxpy(const zd* X, size_t lds, size_t ldv, const int* slot, const int* cnt, const zd* h, double sign,
                       zd* W, size_t n, int A, hipStream_t s);
// x_{slot[a]} (stride n) += sum_{q < cnt[a]} Z_{slot[a], q} y[a*64 + q]
void launch_slincomb(const zd* Z, size_t lds, size_t ldv, const int* slot, const int* cnt, const zd* y, zd* x,
                     size_t n, int A, hipStream_t s);
// Y_a = X_{slot[a], j[a]} (j may be NULL: vector 0)
void launch_sgather(const zd* X, size_t lds, size_t ldv, const int* slot, const int* j, zd* Y, size_t n, int A,
                    hipStream_t s);
// X_{slot[a], j[a]} = c[a] * Y_{src[a]} with Y_k at Y + k*ldy (c NULL: copy; src NULL: a; j NULL: 0)
void launch_sscatter(const zd* Y, size_t ldy, const int* src, zd* X, size_t lds, size_t ldv, const int* slot,
                     const int* j, const double* c, size_t n, int A, hipStream_t s);

// ---- residual.hip: residual norms of the unreduced system (eq. wilson) -------
// relres[r] = ||b_r - D x_r|| / ||b_r|| (||b_r - D x_r|| if b_r = 0) for nrhs
// full-lattice pairs; partial holds 2 * resnorm_nblocks(N) * nrhs doubles,
// relres nrhs doubles (both device)
constexpr int RESNORM_MAX_BLOCKS = 256;
int resnorm_nblocks(int N);
// links from the caller's U[mu][y][x], c = m + 2
void launch_wilson_resnorm(int N, const zd* U, double c, const zd* B, const zd* X, int nrhs, double* partial,
                           double* relres, hipStream_t s);
// links from the hierarchy's packed copy
void launch_wilson_resnorm_packed(const Fine& f, const zd* B, const zd* X, int nrhs, double* partial,
                                  double* relres, hipStream_t s);

// ---- kcycle.hip: the Krylov-accelerated coarse visit of the K-cycle ---------
// Vectors [R][n] (T = double or float), sums and coefficients in FP64;
// coef holds 4 entries per right-hand side (a1, (rho1, 0), beta, a2);
// partial holds kcycle_nblocks(n) * 2 * R complex.
int kcycle_nblocks(size_t n);
// partial sums of <A_r, X1_r> and <A_r, X2_r> (X2 may be NULL)
template <typename T>
void launch_kdots(const cx<T>* A, const cx<T>* X1, const cx<T>* X2, size_t n, int R, zd* partial, hipStream_t s);
// W -= beta W', Z -= beta Z', then the partial sums of <W, W> and <W, X2>
template <typename T>
void launch_korth_dots(cx<T>* W, const cx<T>* Wp, cx<T>* Z, const cx<T>* Zp, const cx<T>* X2, const zd* coef,
                       size_t n, int R, zd* partial, hipStream_t s);
// mode 0: a1 = d2 / Re d1 (and rho1 = Re d1); 1: beta = d1 / rho1; 2: a2 = d2 / Re d1
void launch_kcoef(const zd* partial, size_t n, int R, int mode, zd* coef, hipStream_t s);
// x = a1 z1, r1 = r0 - a1 w1
template <typename T>
void launch_kstep1(const cx<T>* z1, const cx<T>* w1, const cx<T>* r0, const zd* coef, cx<T>* x, cx<T>* r1, size_t n,
                   int R, hipStream_t s);
// x += a2 z2
template <typename T>
void launch_kstep3(const cx<T>* z2, const zd* coef, cx<T>* x, size_t n, int R, hipStream_t s);

// ---- boot.hip: bootstrap multigrid eigensolver (Sec. 3.4, Theorem 1) -------
// lam[r] = <Gamma_5 A v_r, v_r> / <v_r, v_r> for k vectors V with AV = A V
// (dps = 2 on level 0, 16 above); partial holds blas_nblocks(n) * k complex
void launch_ritz(const zd* V, const zd* AV, size_t n, int dps, int k, zd* partial, double* lam, hipStream_t s);
void launch_gamma5(const zd* x, zd* y, size_t n, int dps, int k, hipStream_t s);
// Y_j = sum_i X_i C[i][j], p vectors of length n, C (device) p x p row-major
void launch_block_combine(const zd* X, const zd* C, zd* Y, size_t n, int p, hipStream_t s);
// R_j = A_j - lam_j B_j for k vectors (lam device)
void launch_eig_residual(const zd* A, const zd* B, const double* lam, zd* R, size_t n, int k, hipStream_t s);
// one coarse colour pass on (D - lam_r Gamma_5) x_r = 0 (rows of a site in order)
void launch_kaczmarz_coarse_shift(const Coarse& c, int colour, int mode, int nsites, zd* x, const double* lam,
                                  int nrhs, hipStream_t s);
// P from k (<= 16) test vectors: rank-8 least squares fit per aggregate and spin
// (fine: ex = N/2, ey = N; coarse: the level's site extents)
void launch_fit_ls(bool fine, int ex, int ey, const zd* V, int k, zd* P, hipStream_t s);

}  // namespace bamg
