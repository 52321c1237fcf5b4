// libbamg host side: the C ABI of include/bamg.h, the hierarchy, the
// bootstrap setup, the multigrid cycle and the outer flexible GMRES.
// Every arithmetic step on vectors and operators runs in the HIP kernels of
// fine.hip, coarse.hip, dense.hip and blas.hip; the host orders the launches
// on the hierarchy's stream and performs the O(restart^2) Givens / Hessenberg
// algebra of the Krylov method.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <string>
#include <algorithm>
#include <functional>
#include <vector>

#include "../../include/bamg.h"
#include "bamg_internal.h"
#include "hierarchy.h"

using namespace bamg;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

}  // namespace

int bamg::api_fail(int code, const std::string& msg) { return fail(code, msg); }

namespace {

struct Shape {
  std::vector<std::pair<int, int>> ext;
};

bool level_shapes(const bamg_params* p, Shape& sh, std::string& why) {
  const int N = p->N;
  if (N < 16 || N % 8 != 0) { why = "N must be a multiple of 8 and >= 16"; return false; }
  sh.ext.clear();
  sh.ext.push_back({N / 2, N});
  if (p->n_levels == 1) return true;  // operator only: smoother-preconditioned Krylov
  int ex = N / 8, ey = N / 4;
  sh.ext.push_back({ex, ey});
  while (true) {
    const int L = (int)sh.ext.size();
    if (p->n_levels > 0 && L >= p->n_levels) break;
    if (p->n_levels <= 0 && ex * ey * 16 <= p->max_coarse) break;
    if (ex % 2 || ey % 2 || ex < 4 || ey < 4) break;
    ex /= 2;
    ey /= 2;
    sh.ext.push_back({ex, ey});
  }
  if (p->n_levels > 0 && (int)sh.ext.size() != p->n_levels) { why = "n_levels not reachable for this N"; return false; }
  const size_t nL = (size_t)sh.ext.back().first * sh.ext.back().second * 16;
  if (sh.ext.size() > 1 && nL > 8192) { why = "coarsest level dimension exceeds 8192 (dense inverse); raise n_levels"; return false; }
  return true;
}

bool valid_params(const bamg_params* p, std::string& why) {
  if (!p) { why = "params is NULL"; return false; }
  if (p->n_tv != 8) { why = "n_tv must be 8"; return false; }
  if (p->setup_sweeps < 0 || p->setup_adapt < 0 || p->pre < 0 || p->post < 0) { why = "negative count"; return false; }
  if (p->cycle != BAMG_CYCLE_V && p->cycle != BAMG_CYCLE_W && p->cycle != BAMG_CYCLE_K) { why = "unknown cycle"; return false; }
  if (p->precision < BAMG_FP64 || p->precision > BAMG_MIXED_FP32) { why = "unknown precision"; return false; }
  if (p->restart < 1 || p->restart > 60) { why = "restart must be in [1, 60]"; return false; }
  if (p->max_iter < 0) { why = "max_iter < 0"; return false; }
  if (p->max_coarse < 16) { why = "max_coarse < 16"; return false; }
  if (p->graphs != 0 && p->graphs != 1) { why = "graphs must be 0 or 1"; return false; }
  if (p->setup_mode < 0 || p->setup_mode > 2) { why = "setup_mode must be 0, 1 or 2"; return false; }
  if (p->setup_mode && (p->n_ev < 1 || p->n_ev > 8)) { why = "n_ev must be in [1, 8]"; return false; }
  if (p->setup_mode && (p->boot_nu1 < 0 || p->boot_nu2 < 0)) { why = "negative bootstrap sweep count"; return false; }
  if (p->coarsest_fp32 != 0 && p->coarsest_fp32 != 1) { why = "coarsest_fp32 must be 0 or 1"; return false; }
  if (p->coarsest_fp32 && p->precision == BAMG_FP64) { why = "coarsest_fp32 needs a mixed precision"; return false; }
  if (p->lookahead < 0 || p->lookahead > 2) { why = "lookahead must be 0, 1 or 2"; return false; }
  return true;
}

}  // namespace

// =============================================================================
// C ABI
// =============================================================================
extern "C" {

const char* bamg_last_error(void) { return g_err.c_str(); }

int bamg_default_params(bamg_params* p) {
  if (!p) return fail(BAMG_EINVAL, "params is NULL");
  std::memset(p, 0, sizeof(*p));
  p->N = 0;
  p->n_levels = 0;
  p->max_coarse = 8192;
  p->n_tv = 8;
  p->setup_sweeps = 20;
  p->setup_adapt = 1;
  p->pre = 4;
  p->post = 4;
  p->cycle = BAMG_CYCLE_V;
  p->precision = BAMG_FP64;
  p->restart = 32;
  p->max_iter = 1000;
  p->seed = 0;
  p->init_tv_host = nullptr;
  p->stream = nullptr;
  p->graphs = 0;
  p->setup_mode = 0;
  p->n_ev = 8;
  p->boot_nu1 = 10;
  p->boot_nu2 = 5;
  p->coarsest_fp32 = 0;
  p->lookahead = 1;
  return BAMG_OK;
}

size_t bamg_footprint_bytes(const bamg_params* p) {
  std::string why;
  Shape sh;
  if (!valid_params(p, why) || !level_shapes(p, sh, why)) return 0;
  const size_t N = p->N, k = p->n_tv, z = sizeof(zd);
  const int L = (int)sh.ext.size();
  const bool mg = L > 1, mixed = p->precision != BAMG_FP64;
  const size_t ne = (mg && p->setup_mode) ? p->n_ev : 0;
  const size_t cap = mg ? k + ne : 1;  // right-hand sides of the level work vectors after setup
  const size_t zm = z + (mixed ? sizeof(zf) : 0);  // an entry and its FP32 copy in the mixed modes
  const size_t zc = z + (mixed && p->coarsest_fp32 ? sizeof(zf) : 0);  // entry of the coarsest inverse
  const size_t sst = p->precision == BAMG_MIXED_FP32 ? sizeof(zf) : sizeof(hcx);  // stored coarse operator entry
  auto kvis = [&](int l) { return p->cycle == BAMG_CYCLE_K && l >= 1 && l + 1 < L; };
  size_t bytes = (2 * N * N + (N * N / 2) * 38) * zm;  // links, stored slot blocks of Dhat and their Gram terms
  if (L > 2 && p->cycle == BAMG_CYCLE_K)  // K-cycle reduction partials (the largest visited level is level 1)
    bytes += (size_t)kcycle_nblocks((size_t)sh.ext[1].first * sh.ext[1].second * 16) * 2 * cap * z;
  for (int l = 0; l < L; ++l) {
    const size_t ns = (size_t)sh.ext[l].first * sh.ext[l].second;
    const size_t n = ns * (l == 0 ? 2 : 16);
    const bool last = l == L - 1;
    // x, b, r and, below the coarsest level, the second x of the blocked (level 0) or fused (coarse) sweeps
    bytes += (last && l > 0 ? 3 : 4) * n * cap * zm;
    if (!mg) break;
    if (kvis(l)) bytes += 5 * n * cap * zm + 4 * cap * z;  // K-cycle visit vectors and coefficients
    bytes += n * (k + ne) * z;  // test vectors
    if (l >= 1) bytes += ns * NOFF * 256 * z;  // coarse operator
    if (l >= 1 && !last) bytes += ns * 256 * zm + (mixed ? ns * NOFF * 256 * sst : 0);  // Kinv; stored operator
    if (!last) bytes += n * 8 * zm;  // P
    if (last) {  // inverse, split-K partials, inversion scratch
      bytes += n * n * zc + (dense_mm_workspace((int)n, (int)cap) + gj_workspace((int)n)) * z + n * sizeof(int);
      if (n % 64 == 0) {  // packed gamma5 half of the inverse (and its FP32 copy), block table, partial products
        const size_t nbk = n / 64, nblk = nbk * (nbk + 1) / 2;
        bytes += nblk * 4096 * zc + nblk * 2 * sizeof(int) + 2 * nbk * nbk * 64 * z;
      }
    }
  }
  const size_t n0 = N * N, kd = p->restart;
  if (mg && cap >= (size_t)IL_MIN) bytes += 2 * n0 * cap * zm;  // interleaved level-0 x and b
  bytes += (2 * kd + 5) * n0 * z;  // FGMRES bases and vectors, one right-hand side
  bytes += (size_t)blas_nblocks_fine(n0) * 64 * cap * z;  // reduction partials
  if (mg) bytes += n0 * k * z;     // saved test vectors
  if (ne) {                        // eigensolver blocks
    const size_t nL = (size_t)sh.ext[L - 1].first * sh.ext[L - 1].second * 16, pc = std::min<size_t>(16, nL);
    bytes += (4 * nL * pc + 2 * pc * pc + dense_mm_workspace((int)nL, (int)pc)) * z;
  }
  return bytes;
}

}  // extern "C"

size_t bamg::hierarchy_slot_extra_bytes(const bamg_params* p, int slots) {
  std::string why;
  Shape sh;
  if (!valid_params(p, why) || !level_shapes(p, sh, why) || slots < 1) return 0;
  const int L = (int)sh.ext.size();
  const size_t cap = L > 1 ? p->n_tv + (p->setup_mode ? p->n_ev : 0) : 1;  // as counted by the footprint
  const size_t S = slots;
  if (S <= cap) return 0;
  const size_t zm = sizeof(zd) + (p->precision != BAMG_FP64 ? sizeof(zf) : 0);
  size_t bytes = 0;
  const size_t n0 = (size_t)sh.ext[0].first * sh.ext[0].second * 2;
  if (S >= (size_t)IL_MIN) bytes += 2 * n0 * (S - (cap >= (size_t)IL_MIN ? cap : 0)) * zm;  // interleaved level 0
  if (L > 2 && p->cycle == BAMG_CYCLE_K)
    bytes += (size_t)kcycle_nblocks((size_t)sh.ext[1].first * sh.ext[1].second * 16) * 2 * (S - cap) * sizeof(zd);
  for (int l = 0; l < L; ++l) {
    const size_t n = (size_t)sh.ext[l].first * sh.ext[l].second * (l == 0 ? 2 : 16);
    bytes += (l == L - 1 && l > 0 ? 3 : 4) * n * (S - cap) * zm;  // the level work vectors grow to S right-hand sides
    if (p->cycle == BAMG_CYCLE_K && l >= 1 && l + 1 < L) bytes += (5 * n * zm + 4 * sizeof(zd)) * (S - cap);
    if (l == L - 1 && L > 1)
      bytes += (dense_mm_workspace((int)n, slots) - dense_mm_workspace((int)n, (int)cap)) * sizeof(zd);
  }
  return bytes;
}

extern "C" {

int bamg_setup(const void* gauge, double m, const bamg_params* p, bamg_hierarchy** out) {
  if (!out) return fail(BAMG_EINVAL, "out is NULL");
  *out = nullptr;
  std::string why;
  Shape sh;
  if (!gauge) return fail(BAMG_EINVAL, "gauge is NULL");
  if (!valid_params(p, why) || !level_shapes(p, sh, why)) return fail(BAMG_EINVAL, why);
  if (!std::isfinite(m) || m + 2.0 == 0.0) return fail(BAMG_EINVAL, "mass gives c = m + 2 = 0 or non-finite");
  bamg_hierarchy* h = new bamg_hierarchy();
  try {
    h->p = *p;
    h->p.init_tv_host = nullptr;
    h->m = m;
    h->s = (hipStream_t)p->stream;
    const int N = p->N;
    h->f.N = N;
    h->f.NH = N / 2;
    h->f.c = m + 2.0;
    h->f.kappa = 1.0 / h->f.c;
    h->f.kappa2 = h->f.kappa * h->f.kappa;
    h->Ue = dalloc<zd>((size_t)N * N);
    h->Uo = dalloc<zd>((size_t)N * N);
    h->f.Ue = h->Ue;
    h->f.Uo = h->Uo;
    launch_gauge_pack((const zd*)gauge, h->Ue, h->Uo, N, h->s);
    h->Bst = dalloc<zd>((size_t)N * N / 2 * 36);
    launch_slot_blocks(h->f, h->Bst, h->s);
    h->f.Bst = h->Bst;
    h->Gst = dalloc<zd>((size_t)N * N / 2 * 2);
    launch_slot_gram(h->f, h->Bst, h->Gst, h->s);
    h->f.Gst = h->Gst;
    check_launch();
    const int L = (int)sh.ext.size(), k = p->n_tv;
    const bool mg = L > 1;
    h->lv.resize(L);
    for (int l = 0; l < L; ++l) {
      Level& Lv = h->lv[l];
      Lv.ex = sh.ext[l].first;
      Lv.ey = sh.ext[l].second;
      Lv.dps = (l == 0) ? 2 : 16;
      Lv.n = (size_t)Lv.ex * Lv.ey * Lv.dps;
      if (mg) Lv.tv = dalloc<zd>(Lv.n * (k + (p->setup_mode ? p->n_ev : 0)));
      if (l >= 1) Lv.D = dalloc<zd>((size_t)Lv.ex * Lv.ey * NOFF * 256);
      if (!mg || l < L - 1) {
        h->build_colours(l);
        if (mg) {
          Lv.prow = (l == 0) ? 16 : 32;
          Lv.P = dalloc<zd>(Lv.n * 8);
        }
        if (l >= 1) Lv.Kinv = dalloc<zd>((size_t)Lv.ex * Lv.ey * 256);
      } else {
        Lv.Ainv = dalloc<zd>(Lv.n * Lv.n);
        if (mg && Lv.n % 64 == 0) {  // packed gamma5 half of the inverse for the single-RHS product
          const int nbk = (int)(Lv.n / 64);
          std::vector<int> blk;
          for (int I = 0; I < nbk; ++I)
            for (int J = I; J < nbk; ++J) blk.insert(blk.end(), {I, J});
          Lv.Ablk = dalloc<int>(blk.size());
          HIPCHK(hipMemcpy(Lv.Ablk, blk.data(), blk.size() * sizeof(int), hipMemcpyHostToDevice));
          Lv.Ap = dalloc<zd>(blk.size() / 2 * 64 * 64);
          Lv.Apart = dalloc<zd>((size_t)2 * nbk * nbk * 64);
        }
      }
    }
    h->ensure_cap(mg ? k + (p->setup_mode ? p->n_ev : 0) : 1);
    const size_t n0 = h->lv[0].n;
    h->dflag = dalloc<int>(1);
    HIPCHK(hipHostMalloc((void**)&h->hflag, sizeof(int)));
    h->kdim = p->restart;
    h->ensure_krylov(1, false);
    if (mg) {
      h->gjcol = dalloc<zd>(gj_workspace((int)h->lv.back().n));
      h->gjperm = dalloc<int>(h->lv.back().n);
      h->tvsave = dalloc<zd>(n0 * k);
      // initial test vectors (Sec. 4: random, normal, mean 0, variance 1)
      if (p->init_tv_host) {
        HIPCHK(hipMemcpyAsync(h->lv[0].tv, p->init_tv_host, n0 * k * sizeof(zd), hipMemcpyHostToDevice, h->s));
      } else {
        launch_philox_tv((int)n0, k, p->seed, h->lv[0].tv, h->s);
        check_launch();
      }
      if (p->setup_mode) h->boot_setup();
      else h->setup_pass();
      // adaptive passes: two cycles of the current hierarchy on Dhat v = 0 for
      // every saved level-0 test vector, then relax-fit-coarsen again
      for (int a = 0; a < (p->setup_mode ? 0 : p->setup_adapt); ++a) {
        Level& L0 = h->lv[0];
        launch_copy(h->tvsave, L0.tv, n0 * k, h->s);
        launch_fill_zero(L0.b, n0 * k, h->s);
        for (int c = 0; c < 2; ++c) h->cycle(0, L0.b, L0.tv, k);
        launch_norms(L0.tv, n0, k, n0, h->partial, h->hdev, h->s);
        launch_normalize(L0.tv, n0, k, n0, h->hdev, h->s);
        check_launch();
        h->setup_pass();
      }
    }
    h->refresh_mixed();
    HIPCHK(hipStreamSynchronize(h->s));
  } catch (const HipFail& e) {
    delete h;
    return fail(BAMG_EDEVICE, e.msg);
  } catch (const BadArg& e) {
    delete h;
    return fail(BAMG_ESINGULAR, e.msg);
  }
  *out = h;
  return BAMG_OK;
}

void bamg_free(bamg_hierarchy* h) { delete h; }

int bamg_n_levels(const bamg_hierarchy* h) {
  if (!h) return fail(BAMG_EINVAL, "hierarchy is NULL");
  return h->L();
}

int bamg_level_info(const bamg_hierarchy* h, int32_t l, int32_t* info) {
  if (!h || !info || l < 0 || l >= h->L()) return fail(BAMG_EINVAL, "bad level");
  const Level& Lv = h->lv[l];
  info[0] = Lv.ex;
  info[1] = Lv.ey;
  info[2] = Lv.dps;
  info[3] = (int32_t)Lv.n;
  info[4] = Lv.ncol;
  return BAMG_OK;
}

int bamg_apply_dhat(bamg_hierarchy* h, const void* x, void* y, int32_t nrhs) {
  if (!h || !x || !y || nrhs < 1) return fail(BAMG_EINVAL, "bad arguments");
  if (x == y) return fail(BAMG_EINVAL, "x and y must not alias");
  try {
    h->apply(0, (const zd*)x, (zd*)y, nullptr, nrhs);
  } catch (const HipFail& e) {
    return fail(BAMG_EDEVICE, e.msg);
  }
  return BAMG_OK;
}

int bamg_eo_reduce(bamg_hierarchy* h, const void* b, void* bhat, int32_t nrhs) {
  if (!h || !b || !bhat || nrhs < 1) return fail(BAMG_EINVAL, "bad arguments");
  launch_eo_reduce(h->f, (const zd*)b, (zd*)bhat, nrhs, h->s);
  if (hipGetLastError() != hipSuccess) return fail(BAMG_EDEVICE, "launch failed");
  return BAMG_OK;
}

int bamg_eo_reconstruct(bamg_hierarchy* h, const void* b, const void* xe, void* x, int32_t nrhs) {
  if (!h || !b || !xe || !x || nrhs < 1) return fail(BAMG_EINVAL, "bad arguments");
  launch_eo_reconstruct(h->f, (const zd*)b, (const zd*)xe, (zd*)x, nrhs, h->s);
  if (hipGetLastError() != hipSuccess) return fail(BAMG_EDEVICE, "launch failed");
  return BAMG_OK;
}

int bamg_level_op(bamg_hierarchy* h, int32_t l, int32_t op, const void* in, void* out, int32_t nrhs) {
  if (!h || !in || !out || nrhs < 1 || l < 0 || l >= h->L()) return fail(BAMG_EINVAL, "bad arguments");
  try {
    const zd* xi = (const zd*)in;
    zd* xo = (zd*)out;
    switch (op) {
      case BAMG_OP_APPLY:
        if (in == out) return fail(BAMG_EINVAL, "in and out must not alias");
        h->apply(l, xi, xo, nullptr, nrhs);
        break;
      case BAMG_OP_SWEEP:
        if (h->coarsest(l) && h->L() > 1) return fail(BAMG_EINVAL, "no smoother on the coarsest level");
        if (nrhs > h->cap) h->ensure_cap(nrhs);
        h->smooth(l, xo, xi, nrhs, 1);
        break;
      case BAMG_OP_SWEEP_COLOURS:
        if (h->coarsest(l) && h->L() > 1) return fail(BAMG_EINVAL, "no smoother on the coarsest level");
        h->sweep_colours(l, xo, xi, nrhs);
        break;
      case BAMG_OP_RESTRICT:
        if (h->coarsest(l)) return fail(BAMG_EINVAL, "no restriction from the coarsest level");
        h->restrict_(l, xi, xo, nrhs);
        break;
      case BAMG_OP_PROLONG:
        if (h->coarsest(l)) return fail(BAMG_EINVAL, "no prolongation to the coarsest level");
        h->prolong(l, xi, xo, nrhs);
        break;
      case BAMG_OP_COARSEST:
        if (!h->coarsest(l) || h->L() == 1) return fail(BAMG_EINVAL, "level is not a directly solved coarsest level");
        if (in == out) return fail(BAMG_EINVAL, "in and out must not alias");
        h->ensure_cap(nrhs);  // the split-K product needs workspace for nrhs right-hand sides
        h->coarsest_solve(xi, xo, nrhs);
        break;
      case BAMG_OP_COARSEST_F32: {
        if (!h->c32()) return fail(BAMG_EINVAL, "no FP32 copy of the coarsest inverse (coarsest_fp32 = 0)");
        if (!h->coarsest(l) || h->L() == 1) return fail(BAMG_EINVAL, "level is not a directly solved coarsest level");
        if (in == out) return fail(BAMG_EINVAL, "in and out must not alias");
        h->ensure_cap(nrhs);
        Level& C = h->lv[l];
        if (h->force_mr ||
            !launch_dense_mv_g5_c32(C.Ap32, C.Ablk, (int)C.n, (const zf*)in, (zf*)out, nrhs, C.Apart, h->s))
          launch_dense_mv32(C.Ainv32, (int)C.n, (const zf*)in, (zf*)out, nrhs, h->force_mr, (zf*)h->mmwork, h->s);
        check_launch();
        break;
      }
      case BAMG_OP_CYCLE:
        h->ensure_cap(nrhs);
        launch_fill_zero(xo, h->lv[l].n * nrhs, h->s);
        h->cycle(l, xi, xo, nrhs);
        break;
      case BAMG_OP_RESIDUAL: {
        h->ensure_cap(nrhs);
        Level& Lv = h->lv[l];
        h->apply(l, xo, Lv.r, xi, nrhs);
        launch_copy(Lv.r, xo, Lv.n * nrhs, h->s);
        check_launch();
        break;
      }
      case BAMG_OP_APPLY_MIXED:
      case BAMG_OP_SWEEP_MIXED:
      case BAMG_OP_CYCLE_MIXED:
      case BAMG_OP_APPLY_F32:
      case BAMG_OP_SWEEP_F32:
      case BAMG_OP_SWEEP_COLOURS_F32: {
        if (!h->mixed()) return fail(BAMG_EINVAL, "hierarchy is FP64");
        if (op == BAMG_OP_CYCLE_MIXED) {
          if (l != 0) return fail(BAMG_EINVAL, "the mixed cycle starts on level 0");
          h->ensure_cap(nrhs);
          h->precondition_mixed(xi, xo, nrhs);
          break;
        }
        if ((op == BAMG_OP_SWEEP_MIXED || op == BAMG_OP_SWEEP_F32 || op == BAMG_OP_SWEEP_COLOURS_F32) &&
            h->coarsest(l) && h->L() > 1)
          return fail(BAMG_EINVAL, "no smoother on the coarsest level");
        if (l >= 1 && h->coarsest(l)) return fail(BAMG_EINVAL, "the coarsest level has no smoother; its solve is op 12");
        if (op == BAMG_OP_APPLY_F32 && in == out) return fail(BAMG_EINVAL, "in and out must not alias");
        h->ensure_cap(nrhs);
        Level& Lv = h->lv[l];
        const size_t nn = Lv.n * nrhs;
        const bool f32io = (op == BAMG_OP_APPLY_F32 || op == BAMG_OP_SWEEP_F32 || op == BAMG_OP_SWEEP_COLOURS_F32);
        const bool colours = op == BAMG_OP_SWEEP_COLOURS_F32;
        const bool is_apply = (op == BAMG_OP_APPLY_MIXED || op == BAMG_OP_APPLY_F32);
        // complex64 operands are used in place; complex128 ones go through the level's FP32 vectors
        const zf* bi = f32io ? (const zf*)in : Lv.b32;
        zf* xw = f32io ? (zf*)out : Lv.x32;
        if (!f32io) {
          launch_convert(xi, Lv.b32, nn, h->s);
          if (!is_apply) launch_convert((const zd*)xo, Lv.x32, nn, h->s);
        }
        switch (h->p.precision) {
          case BAMG_MIXED_FP16:
            if (is_apply) h->apply32<hcx>(l, bi, xw, nullptr, nrhs);
            else if (colours) h->sweep_colours32<hcx>(l, xw, bi, nrhs, false);
            else h->smooth32<hcx>(l, xw, bi, nrhs, 1);
            break;
          case BAMG_MIXED_BF16:
            if (is_apply) h->apply32<bcx>(l, bi, xw, nullptr, nrhs);
            else if (colours) h->sweep_colours32<bcx>(l, xw, bi, nrhs, false);
            else h->smooth32<bcx>(l, xw, bi, nrhs, 1);
            break;
          default:
            if (is_apply) h->apply32<zf>(l, bi, xw, nullptr, nrhs);
            else if (colours) h->sweep_colours32<zf>(l, xw, bi, nrhs, false);
            else h->smooth32<zf>(l, xw, bi, nrhs, 1);
            break;
        }
        if (!f32io) launch_convert(Lv.x32, xo, nn, h->s);
        check_launch();
        break;
      }
      default:
        return fail(BAMG_EINVAL, "unknown op");
    }
  } catch (const HipFail& e) {
    return fail(BAMG_EDEVICE, e.msg);
  }
  return BAMG_OK;
}

int bamg_export_level(const bamg_hierarchy* hc, int32_t l, void* P_host, void* Dl_host, void* tv_host) {
  bamg_hierarchy* h = const_cast<bamg_hierarchy*>(hc);
  if (!h || l < 0 || l >= h->L()) return fail(BAMG_EINVAL, "bad level");
  const Level& Lv = h->lv[l];
  try {
    if (P_host) {
      if (!Lv.P) return fail(BAMG_EINVAL, "no P on the coarsest level");
      HIPCHK(hipMemcpyAsync(P_host, Lv.P, Lv.n * 8 * sizeof(zd), hipMemcpyDeviceToHost, h->s));
    }
    if (Dl_host) {
      if (!Lv.D) return fail(BAMG_EINVAL, "level 0 has no block operator");
      HIPCHK(hipMemcpyAsync(Dl_host, Lv.D, (size_t)Lv.ex * Lv.ey * NOFF * 256 * sizeof(zd), hipMemcpyDeviceToHost, h->s));
    }
    if (tv_host) {
      if (l != 0 || !h->tvsave) return fail(BAMG_EINVAL, "test vectors are exported from level 0 of a multigrid hierarchy");
      HIPCHK(hipMemcpyAsync(tv_host, h->tvsave, Lv.n * h->p.n_tv * sizeof(zd), hipMemcpyDeviceToHost, h->s));
    }
    HIPCHK(hipStreamSynchronize(h->s));
  } catch (const HipFail& e) {
    return fail(BAMG_EDEVICE, e.msg);
  }
  return BAMG_OK;
}

int bamg_import_level(bamg_hierarchy* h, int32_t l, const void* P_host, const void* Dl_host) {
  if (!h || l < 0 || l >= h->L() || (!P_host && !Dl_host)) return fail(BAMG_EINVAL, "bad level, or neither P nor D_l");
  if (P_host && l + 1 >= h->L()) return fail(BAMG_EINVAL, "no P on the coarsest level");
  if (Dl_host && (l == 0 || h->L() < 2)) return fail(BAMG_EINVAL, "level 0 has no block operator");
  try {
    Level& Lv = h->lv[l];
    if (Dl_host) {  // D_l replaced: its smoother data, or (coarsest) its inverse, follow
      HIPCHK(hipMemcpyAsync(Lv.D, Dl_host, (size_t)Lv.ex * Lv.ey * NOFF * 256 * sizeof(zd), hipMemcpyHostToDevice,
                            h->s));
      if (h->coarsest(l)) h->invert_coarsest();
      else launch_kaczmarz_prep(Lv.coarse(), Lv.Kinv, h->s);
      check_launch();
    }
    if (P_host) {
      HIPCHK(hipMemcpyAsync(Lv.P, P_host, Lv.n * 8 * sizeof(zd), hipMemcpyHostToDevice, h->s));
      h->build_next(l);
    }
    h->refresh_mixed();
    HIPCHK(hipStreamSynchronize(h->s));
  } catch (const HipFail& e) {
    return fail(BAMG_EDEVICE, e.msg);
  } catch (const BadArg& e) {
    return fail(BAMG_ESINGULAR, e.msg);
  }
  return BAMG_OK;
}

int bamg_boot_op(bamg_hierarchy* h, int32_t l, int32_t op, void* X, double* lam_host, int32_t k) {
  if (!h || !X || !lam_host || k < 1 || l < 0 || l >= h->L()) return fail(BAMG_EINVAL, "bad arguments");
  if (h->L() < 2) return fail(BAMG_EINVAL, "no hierarchy (one level)");
  try {
    h->ensure_boot(8);
    zd* x = (zd*)X;
    switch (op) {
      case BAMG_BOOT_RITZ:
      case BAMG_BOOT_SWEEP:
        if (k > 16) return fail(BAMG_EINVAL, "k > 16");
        h->ensure_cap(k);
        if (op == BAMG_BOOT_SWEEP) {
          if (h->coarsest(l)) return fail(BAMG_EINVAL, "no smoother on the coarsest level");
          HIPCHK(hipMemcpyAsync(h->lam_dev, lam_host, k * sizeof(double), hipMemcpyHostToDevice, h->s));
          h->sweep_shift(l, x, h->lam_dev, k);
        } else {
          h->ritz(l, x, k, h->lam_dev);
          HIPCHK(hipMemcpyAsync(lam_host, h->lam_dev, k * sizeof(double), hipMemcpyDeviceToHost, h->s));
        }
        break;
      case BAMG_BOOT_EIGS: {
        if (!h->coarsest(l)) return fail(BAMG_EINVAL, "eigenpairs are computed on the coarsest level");
        if (k > 8) return fail(BAMG_EINVAL, "k > 8");
        const int ke_save = h->ke;
        const bool he_save = h->have_e;
        h->ke = k;
        h->boot_coarsest(x);
        h->ke = ke_save;
        h->have_e = he_save;
        HIPCHK(hipMemcpyAsync(lam_host, h->lam_dev, k * sizeof(double), hipMemcpyDeviceToHost, h->s));
        break;
      }
      case BAMG_BOOT_FIT: {
        if (h->coarsest(l)) return fail(BAMG_EINVAL, "no interpolation from the coarsest level");
        if (k > 16) return fail(BAMG_EINVAL, "k > 16");
        Level& Lv = h->lv[l];
        if (k <= 8) {
          if (k != h->p.n_tv) return fail(BAMG_EINVAL, "k must be n_tv or in (8, 16]");
          h->fit(l, x);
        } else {
          launch_fit_ls(l == 0, Lv.ex, Lv.ey, x, k, Lv.P, h->s);
          check_launch();
        }
        h->build_next(l);
        h->refresh_mixed();
        break;
      }
      default:
        return fail(BAMG_EINVAL, "unknown op");
    }
    HIPCHK(hipStreamSynchronize(h->s));
  } catch (const HipFail& e) {
    return fail(BAMG_EDEVICE, e.msg);
  } catch (const BadArg& e) {
    return fail(BAMG_ESINGULAR, e.msg);
  }
  return BAMG_OK;
}

int bamg_export_boot(const bamg_hierarchy* hc, double* lam_host, void* ve_host) {
  bamg_hierarchy* h = const_cast<bamg_hierarchy*>(hc);
  if (!h || !lam_host) return fail(BAMG_EINVAL, "bad arguments");
  if (!h->p.setup_mode || !h->have_e) return fail(BAMG_EINVAL, "not a bootstrap hierarchy");
  try {
    for (int k = 0; k < h->ke; ++k) lam_host[k] = h->lam_final[k];
    if (ve_host) {
      HIPCHK(hipMemcpyAsync(ve_host, h->tve(0), h->lv[0].n * h->ke * sizeof(zd), hipMemcpyDeviceToHost, h->s));
      HIPCHK(hipStreamSynchronize(h->s));
    }
  } catch (const HipFail& e) {
    return fail(BAMG_EDEVICE, e.msg);
  }
  return h->ke;
}

int bamg_stationary(bamg_hierarchy* h, void* x, int32_t iters, double* norms_host) {
  if (!h || !x || !norms_host || iters < 0) return fail(BAMG_EINVAL, "bad arguments");
  try {
    h->ensure_krylov(1, true);
    h->ensure_cap(1);
    const size_t n = h->lv[0].n;
    zd* e = (zd*)x;
    hipStream_t s = h->s;
    auto norm_to_host = [&](int i) {
      launch_norms(e, n, 1, n, h->partial, h->hdev, s);
      check_launch();
      HIPCHK(hipMemcpyAsync(h->hhost, h->hdev, sizeof(zd), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      norms_host[i] = std::sqrt(h->hhost[0].x);
    };
    norm_to_host(0);
    for (int it = 0; it < iters; ++it) {
      h->apply(0, e, h->rr, nullptr, 1);  // r = Dhat e (the residual of Dhat e = 0 is -r)
      h->precondition(h->rr, h->w, 1);    // w = M r
      launch_sub(h->w, e, n, s);          // e <- e + M(0 - Dhat e) = e - M r
      norm_to_host(it + 1);
    }
  } catch (const HipFail& e) {
    return fail(BAMG_EDEVICE, e.msg);
  }
  return BAMG_OK;
}

int bamg_full_residual(int32_t N, const void* gauge, double m, const void* B, const void* X, int32_t nrhs,
                       double* relres, void* stream) {
  if (N < 2 || !gauge || !B || !X || !relres || nrhs < 1) return fail(BAMG_EINVAL, "bad arguments");
  hipStream_t s = (hipStream_t)stream;
  double* part = nullptr;
  const size_t bytes = (size_t)2 * resnorm_nblocks(N) * nrhs * sizeof(double);
  if (hipMallocAsync((void**)&part, bytes, s) != hipSuccess) return fail(BAMG_ENOMEM, "partial sums");
  launch_wilson_resnorm(N, (const zd*)gauge, m + 2.0, (const zd*)B, (const zd*)X, nrhs, part, relres, s);
  const hipError_t le = hipGetLastError();
  (void)hipFreeAsync(part, s);
  if (le != hipSuccess) return fail(BAMG_EDEVICE, std::string("launch: ") + hipGetErrorString(le));
  return BAMG_OK;
}

int bamg_fine_sweep_plan(int32_t N, int32_t nrhs, int32_t fp32, int32_t form, int32_t* plan_out) {
  if (!plan_out || N < 1 || nrhs < 1 || form < 0 || form > 3) return fail(BAMG_EINVAL, "bad arguments");
  FineSweepPlan p;
  int sched[3];
  const int got = fine_sweep_plan_query(N, nrhs, fp32 != 0, form, p, sched);
  if (got == 0) return 0;
  int32_t* o = plan_out;
  const int head[9] = {p.Tu, p.Tv, p.ntu, p.ntv, p.i0, p.j0, p.Ru, p.Rv, p.nupd};
  for (int v : head) *o++ = v;
  for (int c = 0; c < 17; ++c) *o++ = p.first[c];
  for (int c = 0; c < 16; ++c) *o++ = p.si0[c];
  for (int c = 0; c < 16; ++c) *o++ = p.sj0[c];
  for (int c = 0; c < 16; ++c) *o++ = p.nj[c];
  for (int k = 0; k < 3; ++k) *o++ = sched[k];
  return got;
}

int bamg_gaussian_tv(int32_t N, int32_t k, uint64_t seed, void* out, void* stream) {
  if (N < 2 || k < 1 || !out) return fail(BAMG_EINVAL, "bad arguments");
  launch_philox_tv(N * N, k, seed, (zd*)out, (hipStream_t)stream);
  if (hipGetLastError() != hipSuccess) return fail(BAMG_EDEVICE, "launch failed");
  return BAMG_OK;
}

// Flexible GMRES(restart), right preconditioned by one cycle (Sec. 4), on the
// reduced systems of R right-hand sides in lockstep: every right-hand side
// has its own Arnoldi basis, Hessenberg matrix and Givens rotations; the
// cycle, the operator and the Gram-Schmidt reductions run batched.  Classical
// Gram-Schmidt applied twice; true residual recomputed at every restart.  A
// right-hand side that stops early keeps zero basis vectors until the others
// finish, so its arithmetic is that of a solve on its own.
// Input: h->bh [R][n]; output: h->xe [R][n], infos[R].
// check_input: a non-finite ||bhat_r|| sends bhat through the finiteness check
// (BAMG_EINVAL if an entry is not finite).  tail (optional): work that
// follows the solve, enqueued with the norms of the true residual whenever
// every right-hand side has passed its estimated-residual test, so that the
// last host round trip covers it; *tail_done says whether it ran (it may run
// on a pass that turns out not to be the last, and then again).
static int fgmres_batch(bamg_hierarchy* h, int R, double tol, bamg_solve_info* infos, bool check_input = false,
                        const std::function<void()>& tail = nullptr, bool* tail_done = nullptr) {
  typedef std::complex<double> C;
  const size_t n = h->lv[0].n;
  const int m = h->kdim;
  hipStream_t s = h->s;
  zd* hh = h->hhost;
  zd* h1 = h->hdev;
  zd* h2 = h->hdev + 64 * R;
  zd* hn2 = h->hdev + 128 * R;
  if (tail_done) *tail_done = false;
  // ||bhat_r||
  launch_norms(h->bh, n, R, n, h->partial, hn2, s, nullptr, true);
  HIPCHK(hipMemcpyAsync(hh, hn2, R * sizeof(zd), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  std::vector<double> bnorm(R), relres(R, 1.0), beta(R);
  std::vector<int> it(R, 0), cycles(R, 0), jend(R, 0);
  std::vector<char> done(R, 0), arn(R, 0);
  bool finite = true;
  for (int r = 0; r < R; ++r) finite = finite && std::isfinite(hh[r].x);
  if (check_input && !finite) {  // an entry that is not finite, or an overflowing norm
    HIPCHK(hipMemsetAsync(h->dflag, 0, sizeof(int), s));
    launch_check_finite(h->bh, n * R, h->dflag, s);
    check_launch();
    HIPCHK(hipMemcpyAsync(h->hflag, h->dflag, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (*h->hflag) return fail(BAMG_EINVAL, "right-hand side is not finite");
  }
  for (int r = 0; r < R; ++r) {
    bnorm[r] = std::sqrt(hh[r].x);
    if (bnorm[r] == 0.0) { done[r] = 1; relres[r] = 0.0; }
  }
  launch_fill_zero(h->xe, n * R, s);
  std::vector<C> H((size_t)R * (m + 1) * m), g((size_t)R * (m + 1)), sn((size_t)R * m);
  std::vector<double> cs((size_t)R * m);
  // the first pass starts from x = 0: its residual is bhat, whose norms are
  // already on the host (the same kernel on the same vector)
  bool first = true, settled = false;
  while (true) {
    const zd* res = first ? h->bh : h->rr;
    if (!first) {
      launch_norms(h->rr, n, R, n, h->partial, hn2, s, nullptr, true);
      HIPCHK(hipMemcpyAsync(hh, hn2, R * sizeof(zd), hipMemcpyDeviceToHost, s));
      if (tail && settled) {
        tail();
        if (tail_done) *tail_done = true;
      }
      HIPCHK(hipStreamSynchronize(s));
    }
    first = false;
    bool any = false;
    for (int r = 0; r < R; ++r) {
      arn[r] = 0;
      if (done[r] && bnorm[r] == 0.0) continue;
      beta[r] = std::sqrt(hh[r].x);
      relres[r] = beta[r] / bnorm[r];
      if (!(relres[r] > tol) || it[r] >= h->p.max_iter) done[r] = 1;
      if (!done[r]) {
        arn[r] = 1;
        any = true;
        ++cycles[r];
      }
      jend[r] = 0;
      h->scal_host[r] = arn[r] ? 1.0 / beta[r] : 0.0;
      std::fill(g.begin() + (size_t)r * (m + 1), g.begin() + (size_t)(r + 1) * (m + 1), C(0.0));
      std::fill(H.begin() + (size_t)r * (m + 1) * m, H.begin() + (size_t)(r + 1) * (m + 1) * m, C(0.0));
      g[(size_t)r * (m + 1)] = arn[r] ? beta[r] : 0.0;
    }
    if (!any) break;
    if (tail_done) *tail_done = false;
    HIPCHK(hipMemcpyAsync(h->scal_dev, h->scal_host, R * sizeof(double), hipMemcpyHostToDevice, s));
    launch_bscale(res, h->V, n, R, h->scal_dev, s);
    int jmax = 0;
    settled = true;
    // iteration j: z_j = M v_j, w = Dhat z_j, CGS2 against v_0..v_j, |w|^2,
    // the results to the host (one right-hand side: the results of odd j in
    // the second set, and v_{j+1} = w / |w| formed on the device from the
    // norm at the end, used or not)
    auto iterate = [&](int j) {
      zd* vj = h->V + (size_t)j * R * n;
      zd* zj = h->Z + (size_t)j * R * n;
      zd* vnext = h->V + (size_t)(j + 1) * R * n;  // (the basis holds m + 1 vectors)
      const size_t o = (R == 1 && (j & 1)) ? HSET1 : 0;
      h->run_graph(((uint64_t)R << 8) | (uint64_t)j, [&] {
        hipStream_t sc = h->s;
        h->precondition(vj, zj, R);
        if (baxpy_dot_applies(n)) {
          // the second projection's inner products and the norm ride on the
          // multi-axpys before them; the reductions also write their results
          // to the pinned host copy themselves (no copy after them); one
          // right-hand side: the norm's reduction also scales w into v_{j+1}
          h->apply(0, zj, h->w, nullptr, R);
          launch_bmultidot(h->V, j + 1, h->w, n, R, h->partial, h1 + o, sc, hh + o);
          launch_baxpy_dot(h->V, j + 1, h1 + o, -1.0, h->w, n, R, j + 1, h->partial, h2 + o, sc, hh + o + 64 * R);
          if (R == 1) {
            launch_baxpy_dot(h->V, j + 1, h2 + o, -1.0, h->w, n, R, 0, h->partial, nullptr, sc);
            launch_norm_scale(h->partial, h->w, vnext, n, hn2 + o, hh + o + 128, sc);
          } else {
            launch_baxpy_dot(h->V, j + 1, h2 + o, -1.0, h->w, n, R, 0, h->partial, hn2 + o, sc, hh + o + 128 * R);
          }
          check_launch();
        } else {
          h->apply(0, zj, h->w, nullptr, R);
          launch_bmultidot(h->V, j + 1, h->w, n, R, h->partial, h1 + o, sc);
          launch_bmultiaxpy(h->V, j + 1, h1 + o, -1.0, h->w, n, R, sc);
          launch_bmultidot(h->V, j + 1, h->w, n, R, h->partial, h2 + o, sc);
          launch_bmultiaxpy(h->V, j + 1, h2 + o, -1.0, h->w, n, R, sc);
          launch_norms(h->w, n, R, n, h->partial, hn2 + o, sc, nullptr, true);
          if (R == 1) launch_bscale_rnorm(h->w, vnext, n, hn2 + o, sc);
          check_launch();
          HIPCHK(hipMemcpyAsync(hh + o, h->hdev + o, (size_t)(128 * R + R) * sizeof(zd), hipMemcpyDeviceToHost, sc));
        }
      });
    };
    bool queued = false;  // iteration j already on the stream (look-ahead)
    for (int j = 0; j < m; ++j) {
      if (!queued) iterate(j);
      // look-ahead (one right-hand side): queue iteration j + 1 before
      // reading j's results when j is unlikely to end the solve; it only
      // needs what j leaves on the device
      queued = R == 1 && h->p.lookahead && j + 1 < m && it[0] + 1 < h->p.max_iter &&
               (h->p.lookahead == 2 || std::abs(g[j]) > 1000.0 * tol * bnorm[0]);
      if (queued) {
        if (!h->ev_iter) HIPCHK(hipEventCreateWithFlags(&h->ev_iter, hipEventDisableTiming));
        HIPCHK(hipEventRecord(h->ev_iter, s));
        iterate(j + 1);
        HIPCHK(hipEventSynchronize(h->ev_iter));
      } else {
        HIPCHK(hipStreamSynchronize(s));
      }
      const zd* hj = hh + ((R == 1 && (j & 1)) ? HSET1 : 0);
      jmax = j + 1;
      bool still = false;
      for (int r = 0; r < R; ++r) {
        h->scal_host[r] = 0.0;
        if (!arn[r]) continue;
        C* Hr = &H[(size_t)r * (m + 1) * m];
        C* gr = &g[(size_t)r * (m + 1)];
        C* snr = &sn[(size_t)r * m];
        double* csr = &cs[(size_t)r * m];
        for (int q = 0; q <= j; ++q)
          Hr[(size_t)q * m + j] = C(hj[r * 64 + q].x, hj[r * 64 + q].y) + C(hj[64 * R + r * 64 + q].x, hj[64 * R + r * 64 + q].y);
        const double hn = std::sqrt(hj[128 * R + r].x);
        if (!std::isfinite(hn)) throw HipFail("non-finite Arnoldi vector");
        for (int q = 0; q < j; ++q) {
          const C a = Hr[(size_t)q * m + j], bq = Hr[(size_t)(q + 1) * m + j];
          Hr[(size_t)q * m + j] = csr[q] * a + snr[q] * bq;
          Hr[(size_t)(q + 1) * m + j] = -std::conj(snr[q]) * a + csr[q] * bq;
        }
        const C a = Hr[(size_t)j * m + j];
        const double aa = std::abs(a);
        double c;
        C sv;
        if (hn == 0.0) { c = 1.0; sv = 0.0; }
        else if (aa == 0.0) { c = 0.0; sv = 1.0; }
        else {
          const double t = std::sqrt(aa * aa + hn * hn);
          c = aa / t;
          sv = (a / aa) * (hn / t);
        }
        csr[j] = c;
        snr[j] = sv;
        Hr[(size_t)j * m + j] = c * a + sv * hn;
        gr[j + 1] = -std::conj(sv) * gr[j];
        gr[j] = c * gr[j];
        ++it[r];
        jend[r] = j + 1;
        if (std::abs(gr[j + 1]) <= tol * bnorm[r] || it[r] >= h->p.max_iter || hn == 0.0) {
          arn[r] = 0;
          if (!(std::abs(gr[j + 1]) <= tol * bnorm[r]) && it[r] < h->p.max_iter) settled = false;
        } else {
          h->scal_host[r] = 1.0 / hn;
          still = true;
        }
      }
      if (!still) break;
      if (j + 1 == m) settled = false;  // a restart follows
      if (R > 1) {
        HIPCHK(hipMemcpyAsync(h->scal_dev, h->scal_host, R * sizeof(double), hipMemcpyHostToDevice, s));
        launch_bscale(h->w, h->V + (size_t)(j + 1) * R * n, n, R, h->scal_dev, s);
      }
    }
    // y_r = H_r^{-1} g_r (upper triangular), x_r += Z_r y_r, true residual
    for (int r = 0; r < R; ++r) {
      zd* yc = h->ycoef_host + (size_t)r * 64;
      for (int q = 0; q < 64; ++q) yc[q] = zd{0, 0};
      const C* Hr = &H[(size_t)r * (m + 1) * m];
      const C* gr = &g[(size_t)r * (m + 1)];
      std::vector<C> y(jend[r]);
      for (int i = jend[r] - 1; i >= 0; --i) {
        C sum = gr[i];
        for (int q = i + 1; q < jend[r]; ++q) sum -= Hr[(size_t)i * m + q] * y[q];
        y[i] = sum / Hr[(size_t)i * m + i];
      }
      for (int q = 0; q < jend[r]; ++q) yc[q] = zd{y[q].real(), y[q].imag()};
    }
    HIPCHK(hipMemcpyAsync(h->ycoef_dev, h->ycoef_host, (size_t)64 * R * sizeof(zd), hipMemcpyHostToDevice, s));
    launch_blincomb(h->Z, jmax, h->ycoef_dev, h->xe, n, R, s);
    h->apply(0, h->xe, h->rr, h->bh, R);
  }
  int worst = BAMG_OK;
  for (int r = 0; r < R; ++r) {
    infos[r].iters = it[r];
    infos[r].restarts = cycles[r] > 0 ? cycles[r] - 1 : 0;
    infos[r].relres_reduced = relres[r];
    infos[r].relres_full = 0.0;
    infos[r].rho_est = it[r] > 0 ? std::pow(relres[r], 1.0 / it[r]) : 0.0;
    if (relres[r] > tol) worst = BAMG_NOT_CONVERGED;
  }
  return worst;
}

static int solve_single(bamg_hierarchy* h, const void* B, void* X, double tol, bamg_solve_info* info) {
  const auto t0 = std::chrono::steady_clock::now();
  int st;
  try {
    h->ensure_krylov(1, true);
    h->ensure_cap(1);
    launch_eo_reduce(h->f, (const zd*)B, h->bh, 1, h->s);
    // x_o from x_e, and ||b - D x|| / ||b|| of the unreduced system (one
    // apply of D and two norms), into a slot of hdev / hhost the Krylov
    // solver does not use (past h1, h2 and |w|^2)
    zd* rf_dev = h->hdev + 129;
    zd* rf_host = h->hhost + 129;
    auto tail = [&] {
      launch_eo_reconstruct(h->f, (const zd*)B, h->xe, (zd*)X, 1, h->s);
      launch_wilson_resnorm_packed(h->f, (const zd*)B, (const zd*)X, 1, (double*)h->partial, (double*)rf_dev, h->s);
      check_launch();
      HIPCHK(hipMemcpyAsync(rf_host, rf_dev, sizeof(double), hipMemcpyDeviceToHost, h->s));
    };
    bool tail_done = false;
    st = fgmres_batch(h, 1, tol, info, true, tail, &tail_done);
    if (st == BAMG_EINVAL) return st;
    if (!tail_done) tail();
    HIPCHK(hipStreamSynchronize(h->s));
    info->relres_full = ((const double*)rf_host)[0];
  } catch (const HipFail& e) {
    return fail(BAMG_EDEVICE, e.msg);
  }
  info->t_solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (st == BAMG_NOT_CONVERGED) g_err = "not converged within max_iter";
  return st;
}

// R right-hand sides through the slot engine, all admitted at once
static int solve_batched(bamg_hierarchy* h, const void* B, void* X, int R, double tol, bamg_solve_info* infos) {
  const auto t0 = std::chrono::steady_clock::now();
  int worst = BAMG_OK;
  try {
    const size_t n = h->lv[0].n;
    HIPCHK(hipMemsetAsync(h->dflag, 0, sizeof(int), h->s));
    launch_check_finite((const zd*)B, 2 * n * R, h->dflag, h->s);
    check_launch();
    HIPCHK(hipMemcpyAsync(h->hflag, h->dflag, sizeof(int), hipMemcpyDeviceToHost, h->s));
    HIPCHK(hipStreamSynchronize(h->s));
    if (*h->hflag) return fail(BAMG_EINVAL, "right-hand side is not finite");
    if (h->engine && engine_capacity(h->engine) < R) {
      engine_destroy(h->engine);
      h->engine = nullptr;
    }
    if (!h->engine) h->engine = engine_create(h, R);
    SlotEngine* e = h->engine;
    for (int r = 0; r < R; ++r)
      engine_admit(e, (const zd*)B + (size_t)r * 2 * n, (zd*)X + (size_t)r * 2 * n, tol, (uint64_t)r);
    std::vector<SlotDone> done;
    while (engine_busy(e) > 0) {
      engine_issue_pre(e);
      engine_finish_pre(e);
      engine_issue_main(e);
      engine_finish_main(e, done);
    }
    for (const SlotDone& d : done) {
      infos[d.tag] = d.info;
      if (d.status == BAMG_EDEVICE) worst = BAMG_EDEVICE;
      else if (d.status != BAMG_OK && worst == BAMG_OK) worst = d.status;
    }
  } catch (const HipFail& e) {
    // the engine may hold slots of this call: drop it (rebuilt on the next call)
    (void)hipStreamSynchronize(h->s);
    if (h->engine) engine_destroy(h->engine);
    h->engine = nullptr;
    return fail(BAMG_EDEVICE, e.msg);
  }
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  for (int r = 0; r < R; ++r) infos[r].t_solve_ms = ms;
  if (worst == BAMG_NOT_CONVERGED) g_err = "not converged within max_iter";
  if (worst == BAMG_EDEVICE) return fail(BAMG_EDEVICE, "non-finite Arnoldi vector");
  return worst;
}

int bamg_solve(bamg_hierarchy* h, const void* b, void* x, double tol, bamg_solve_info* info) {
  if (!h || !b || !x) return fail(BAMG_EINVAL, "bad arguments");
  if (!(tol > 0)) return fail(BAMG_EINVAL, "tol must be > 0");
  bamg_solve_info tmp{};
  if (!info) info = &tmp;
  *info = bamg_solve_info{};
  return solve_single(h, b, x, tol, info);
}

int bamg_solve_batch(bamg_hierarchy* h, const void* B, void* X, int32_t nrhs, double tol, bamg_solve_info* infos) {
  if (!h || !B || !X || nrhs < 1) return fail(BAMG_EINVAL, "bad arguments");
  if (!(tol > 0)) return fail(BAMG_EINVAL, "tol must be > 0");
  if (nrhs > 4096) return fail(BAMG_EINVAL, "nrhs > 4096");
  std::vector<bamg_solve_info> tmp;
  if (!infos) {
    tmp.resize(nrhs);
    infos = tmp.data();
  }
  for (int r = 0; r < nrhs; ++r) infos[r] = bamg_solve_info{};
  return solve_batched(h, B, X, nrhs, tol, infos);
}

}  // extern "C"
