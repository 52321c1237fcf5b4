// Residual of the unreduced system (Sec. 2, eq. wilson): for nrhs full-lattice
// pairs (b, x), relres[r] = ||b_r - D x_r|| / ||b_r|| with D = (m + 2) I - H
// (||b_r - D x_r|| where b_r = 0).  One thread per lattice site forms (D x)(z)
// from the four hops of eq. (wilson), each a rank-one projector times a link
// (P_mu^{+-} = (I +- gamma_mu)/2, gamma_1 = [[0,1],[1,0]], gamma_2 = [[0,i],[-i,0]]);
// the squares are summed per work-group in a fixed tree order and the
// work-groups' sums in a fixed order by one more launch, so the result is
// deterministic.  Links are read from the caller's U[mu][y][x] array or from
// the hierarchy's even/odd packed copy.
#include <mutex>
#include <string>

#include "../../include/bamg.h"
#include "bamg_internal.h"

namespace bamg {
int api_fail(int code, const std::string& msg);

namespace {

constexpr int RT = 256;  // threads per work-group

// U[mu][y][x] as the caller passes it
struct LinksAbi {
  const zd* U;
  int N;
  __device__ __forceinline__ zd at(int mu, int x, int y) const { return U[((size_t)mu * N + y) * N + x]; }
};
// the hierarchy's packed links: the two forward links of the even (odd) site
// with half-x index (xh, y) at Ue (Uo)[(y N/2 + xh) 2 + mu]
struct LinksPacked {
  const zd* Ue;
  const zd* Uo;
  int N;
  __device__ __forceinline__ zd at(int mu, int x, int y) const {
    const size_t i = ((size_t)y * (N >> 1) + (x >> 1)) * 2 + mu;
    return ((x + y) & 1) ? Uo[i] : Ue[i];
  }
};

__device__ __forceinline__ int wrap(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

// partial[(r nb + b) 2 + 0 / 1] = sum over the sites of chunk b of |b - D x|^2 / |b|^2
template <typename Links>
__global__ __launch_bounds__(RT) void k_wilson_resnorm(Links lk, int N, double c, const zd* __restrict__ B,
                                                       const zd* __restrict__ X, double* __restrict__ partial) {
  __shared__ double sh[2 * RT];
  const int blk = blockIdx.x, r = blockIdx.y, nb = gridDim.x, tid = threadIdx.x;
  const size_t sites = (size_t)N * N;
  const size_t chunk = (sites + nb - 1) / nb;
  const size_t lo = (size_t)blk * chunk, hi = (lo + chunk < sites) ? lo + chunk : sites;
  const zd* b = B + (size_t)r * 2 * sites;
  const zd* x = X + (size_t)r * 2 * sites;
  double rr = 0.0, bb = 0.0;
  for (size_t q = lo + tid; q < hi; q += RT) {
    const int y = (int)(q / N), xx = (int)(q - (size_t)y * N);
    const int xp = wrap(xx + 1, N), xm = wrap(xx - 1, N), yp = wrap(y + 1, N), ym = wrap(y - 1, N);
    zd o0 = {0, 0}, o1 = {0, 0}, h;
    // +x: P_1^- U_1(z) psi(z + 1): h = u (a - b) -> (h, -h)
    {
      const zd u = lk.at(0, xx, y), a = x[((size_t)y * N + xp) * 2], bv = x[((size_t)y * N + xp) * 2 + 1];
      h = u * (a - bv);
      o0 = o0 + h;
      o1 = o1 - h;
    }
    // -x: P_1^+ conj(U_1(z - 1)) psi(z - 1): h = u (a + b) -> (h, h)
    {
      const zd u = conj(lk.at(0, xm, y)), a = x[((size_t)y * N + xm) * 2], bv = x[((size_t)y * N + xm) * 2 + 1];
      h = u * (a + bv);
      o0 = o0 + h;
      o1 = o1 + h;
    }
    // +y: P_2^- U_2(z) psi(z + 2): h = u (a - i b) -> (h, i h)
    {
      const zd u = lk.at(1, xx, y), a = x[((size_t)yp * N + xx) * 2], bv = x[((size_t)yp * N + xx) * 2 + 1];
      h = u * (a - mul_i(bv));
      o0 = o0 + h;
      o1 = o1 + mul_i(h);
    }
    // -y: P_2^+ conj(U_2(z - 2)) psi(z - 2): h = u (a + i b) -> (h, -i h)
    {
      const zd u = conj(lk.at(1, xx, ym)), a = x[((size_t)ym * N + xx) * 2], bv = x[((size_t)ym * N + xx) * 2 + 1];
      h = u * (a + mul_i(bv));
      o0 = o0 + h;
      o1 = o1 - mul_i(h);
    }
    const zd x0 = x[q * 2], x1 = x[q * 2 + 1], b0 = b[q * 2], b1 = b[q * 2 + 1];
    // (D x)(z) = c x(z) - (1/2) (o0, o1)
    const zd r0 = b0 - (c * x0 - 0.5 * o0), r1 = b1 - (c * x1 - 0.5 * o1);
    rr += norm2(r0) + norm2(r1);
    bb += norm2(b0) + norm2(b1);
  }
  sh[tid] = rr;
  sh[RT + tid] = bb;
  __syncthreads();
  for (int off = RT / 2; off > 0; off >>= 1) {
    if (tid < off) {
      sh[tid] += sh[tid + off];
      sh[RT + tid] += sh[RT + tid + off];
    }
    __syncthreads();
  }
  if (tid == 0) {
    partial[((size_t)r * nb + blk) * 2] = sh[0];
    partial[((size_t)r * nb + blk) * 2 + 1] = sh[RT];
  }
}

__global__ __launch_bounds__(RT) void k_resnorm_final(const double* __restrict__ partial, int nb,
                                                      double* __restrict__ relres) {
  __shared__ double sh[2 * RT];
  const int r = blockIdx.x, tid = threadIdx.x;
  double rr = 0.0, bb = 0.0;
  for (int b = tid; b < nb; b += RT) {
    rr += partial[((size_t)r * nb + b) * 2];
    bb += partial[((size_t)r * nb + b) * 2 + 1];
  }
  sh[tid] = rr;
  sh[RT + tid] = bb;
  __syncthreads();
  for (int off = RT / 2; off > 0; off >>= 1) {
    if (tid < off) {
      sh[tid] += sh[tid + off];
      sh[RT + tid] += sh[RT + tid + off];
    }
    __syncthreads();
  }
  if (tid == 0) relres[r] = sh[RT] > 0.0 ? sqrt(sh[0] / sh[RT]) : sqrt(sh[0]);
}

}  // namespace

int resnorm_nblocks(int N) {
  const size_t sites = (size_t)N * N;
  size_t nb = (sites + 1023) / 1024;
  if (nb < 1) nb = 1;
  if (nb > RESNORM_MAX_BLOCKS) nb = RESNORM_MAX_BLOCKS;
  return (int)nb;
}

void launch_wilson_resnorm(int N, const zd* U, double c, const zd* B, const zd* X, int nrhs, double* partial,
                           double* relres, hipStream_t s) {
  const int nb = resnorm_nblocks(N);
  hipLaunchKernelGGL(k_wilson_resnorm<LinksAbi>, dim3(nb, nrhs), dim3(RT), 0, s, LinksAbi{U, N}, N, c, B, X, partial);
  hipLaunchKernelGGL(k_resnorm_final, dim3(nrhs), dim3(RT), 0, s, (const double*)partial, nb, relres);
}

void launch_wilson_resnorm_packed(const Fine& f, const zd* B, const zd* X, int nrhs, double* partial,
                                  double* relres, hipStream_t s) {
  const int nb = resnorm_nblocks(f.N);
  hipLaunchKernelGGL(k_wilson_resnorm<LinksPacked>, dim3(nb, nrhs), dim3(RT), 0, s, LinksPacked{f.Ue, f.Uo, f.N},
                     f.N, f.c, B, X, partial);
  hipLaunchKernelGGL(k_resnorm_final, dim3(nrhs), dim3(RT), 0, s, (const double*)partial, nb, relres);
}

// ---------------------------------------------------------------------------
// The same residual norms with no allocation: the partial sums live in a
// file-scope device array, one copy per GPU, held until the process ends.
// Host code never passes the array's name to a kernel (on the host it is a
// stand-in, not a device address): the first call on a device looks up that
// device's copy with hipGetSymbolAddress and keeps the pointer.  Every
// partial sum is written before it is read, so nothing needs clearing; calls
// that overlap on one GPU share the array and race.
// ---------------------------------------------------------------------------
constexpr size_t RESNORM_SCRATCH_DOUBLES = (size_t)1 << 17;  // 1 MiB
static __device__ __align__(256) double scratch[RESNORM_SCRATCH_DOUBLES];

namespace {
std::mutex g_scratch_mu;
constexpr int MAX_DEVICES = 64;
double* g_scratch_ptr[MAX_DEVICES] = {};

// this device's copy of `scratch`, looked up once per device (NULL on failure)
double* scratch_of_current_device(std::string& why) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
    why = "no current HIP device";
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      why = std::string("hipGetSymbolAddress: ") + hipGetErrorString(e);
      return nullptr;
    }
    g_scratch_ptr[dev] = (double*)ptr;
  }
  return g_scratch_ptr[dev];
}
}  // namespace

}  // namespace bamg

extern "C" int bamg_full_residual_noalloc(int32_t N, const void* gauge, double m, const void* B, const void* X,
                                          int32_t nrhs, double* relres, void* stream) {
  using namespace bamg;
  if (N < 2 || !gauge || !B || !X || !relres || nrhs < 1) return api_fail(BAMG_EINVAL, "bad arguments");
  const size_t need = (size_t)2 * resnorm_nblocks(N) * nrhs;
  if (need > RESNORM_SCRATCH_DOUBLES)
    return api_fail(BAMG_EINVAL, "partial sums of " + std::to_string(need) + " doubles exceed the " +
                                     std::to_string(RESNORM_SCRATCH_DOUBLES) + " of the static scratch");
  std::string why;
  double* part = scratch_of_current_device(why);
  if (!part) return api_fail(BAMG_EDEVICE, why);
  launch_wilson_resnorm(N, (const zd*)gauge, m + 2.0, (const zd*)B, (const zd*)X, nrhs, part, relres,
                        (hipStream_t)stream);
  const hipError_t le = hipGetLastError();
  if (le != hipSuccess) return api_fail(BAMG_EDEVICE, std::string("launch: ") + hipGetErrorString(le));
  return BAMG_OK;
}
