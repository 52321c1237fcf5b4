// Slot-based flexible GMRES (FP64, restart m, CGS2 Arnoldi, Givens on the
// host; Sec. 4 uses GMRES(32) preconditioned by the multigrid cycle) for many
// right-hand sides of one hierarchy that enter and leave independently.
//
// Each slot holds one right-hand side: its reduced right-hand side bhat, its
// iterate x_e, its residual, its Arnoldi basis V (m+1 vectors) and its
// preconditioned directions Z (m vectors), all slot-major.  A round advances
// every slot in the Arnoldi phase by one iteration: the current basis vectors
// are gathered into a contiguous block, the cycle and Dhat run on that block
// with the multi-RHS kernels, and the Gram-Schmidt products use the
// slot-mapped kernels.  Slots that finish a restart cycle update x_e, form the
// true residual and re-enter through the norm phase of the next round; new
// right-hand sides enter through the same phase.  Every kernel treats the
// entries of a launch independently with a fixed reduction order, so a
// right-hand side's result is bitwise the same whatever else is in flight.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdint>
#include <cstring>

#include "hierarchy.h"

namespace bamg {

namespace {

typedef std::complex<double> C;

enum SlotState { FREE = 0, NEW, RESTART, ARNOLDI, FINISHING };

struct Slot {
  int state = FREE;
  uint64_t tag = 0;
  const zd* B = nullptr;
  zd* X = nullptr;
  double tol = 0, bnorm = 0, beta = 0, relres = 1;
  int it = 0, cycles = 0, j = 0, status = BAMG_OK;
  bool reconstructed = false;  // x written and its full-system residual queued
  std::chrono::steady_clock::time_point t0;
  std::vector<C> H, g, sn;
  std::vector<double> cs;
};

// index and coefficient arrays uploaded for one phase of a round
constexpr int NI = 8;  // int arrays of `slots` entries per phase
enum Phase { PH_PRE = 0, PH_START, PH_MAIN, PH_POST, NPH };

}  // namespace

struct SlotEngine {
  bamg_hierarchy* h = nullptr;
  int S = 0, m = 0;
  size_t n = 0;
  zd *V = nullptr, *Z = nullptr, *bh = nullptr, *xe = nullptr, *rr = nullptr;
  zd *cur = nullptr, *zc = nullptr, *w = nullptr;
  zd *partial = nullptr, *hdev = nullptr, *hhost = nullptr;  // [4][S][64]
  int *flag_dev = nullptr, *flag_host = nullptr;              // [S][2]: non-finite input
  // full-system residual of each finished slot: partial sums [S][2 RESNORM_MAX_BLOCKS], result [S]
  double *rpart = nullptr, *rf_dev = nullptr, *rf_host = nullptr;
  // per phase: NI int arrays [S], one double array [S], y coefficients [S][64]
  int *ih = nullptr, *id = nullptr;
  double *ch = nullptr, *cd = nullptr;
  zd *yh = nullptr, *yd = nullptr;
  std::vector<Slot> slots;
  std::vector<int> pre_list, act, finishing;
  int busy = 0;

  int* ihost(int ph, int k) { return ih + ((size_t)ph * NI + k) * S; }
  int* idev(int ph, int k) { return id + ((size_t)ph * NI + k) * S; }
  double* chost(int ph) { return ch + (size_t)ph * S; }
  double* cdev(int ph) { return cd + (size_t)ph * S; }
  // upload the first `ni` int arrays (K entries each), the doubles and `ny` y rows of phase ph
  void upload(int ph, int ni, int K, bool coef, int ny) {
    hipStream_t s = h->s;
    for (int k = 0; k < ni; ++k)
      HIPCHK(hipMemcpyAsync(idev(ph, k), ihost(ph, k), (size_t)K * sizeof(int), hipMemcpyHostToDevice, s));
    if (coef) HIPCHK(hipMemcpyAsync(cdev(ph), chost(ph), (size_t)K * sizeof(double), hipMemcpyHostToDevice, s));
    if (ny > 0) HIPCHK(hipMemcpyAsync(yd, yh, (size_t)ny * 64 * sizeof(zd), hipMemcpyHostToDevice, s));
  }

  ~SlotEngine() {
    dfree(V); dfree(Z); dfree(bh); dfree(xe); dfree(rr); dfree(cur); dfree(zc); dfree(w);
    dfree(partial); dfree(hdev); dfree(flag_dev); dfree(id); dfree(cd); dfree(yd);
    dfree(rpart); dfree(rf_dev);
    if (rf_host) (void)hipHostFree(rf_host);
    if (hhost) (void)hipHostFree(hhost);
    if (flag_host) (void)hipHostFree(flag_host);
    if (ih) (void)hipHostFree(ih);
    if (ch) (void)hipHostFree(ch);
    if (yh) (void)hipHostFree(yh);
  }

  void finish_slot(int s, std::vector<SlotDone>& done) {
    Slot& sl = slots[s];
    SlotDone d;
    d.tag = sl.tag;
    d.status = sl.status;
    if (d.status == BAMG_OK && sl.relres > sl.tol) d.status = BAMG_NOT_CONVERGED;
    d.info = bamg_solve_info{};
    d.info.iters = sl.it;
    d.info.restarts = sl.cycles > 0 ? sl.cycles - 1 : 0;
    d.info.relres_reduced = sl.relres;
    d.info.relres_full = sl.reconstructed ? rf_host[s] : 0.0;
    d.info.rho_est = sl.it > 0 ? std::pow(sl.relres, 1.0 / sl.it) : 0.0;
    d.info.t_solve_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - sl.t0).count();
    done.push_back(d);
    sl = Slot{};
    --busy;
  }
};

size_t engine_slot_bytes(size_t n0, int restart, int slots) {
  const size_t z = sizeof(zd);
  return (size_t)slots * n0 * z * (size_t)(2 * restart + 1 + 6) + (size_t)blas_nblocks(n0) * 64 * slots * z +
         (size_t)4 * 64 * slots * z + (size_t)(2 * RESNORM_MAX_BLOCKS + 1) * slots * sizeof(double);
}

SlotEngine* engine_create(bamg_hierarchy* h, int S) {
  SlotEngine* e = new SlotEngine();
  try {
    e->h = h;
    e->S = S;
    e->m = h->kdim;
    e->n = h->lv[0].n;
    const size_t n = e->n, m = e->m;
    e->V = dalloc<zd>((size_t)S * (m + 1) * n);
    e->Z = dalloc<zd>((size_t)S * m * n);
    e->bh = dalloc<zd>((size_t)S * n);
    e->xe = dalloc<zd>((size_t)S * n);
    e->rr = dalloc<zd>((size_t)S * n);
    e->cur = dalloc<zd>((size_t)S * n);
    e->zc = dalloc<zd>((size_t)S * n);
    e->w = dalloc<zd>((size_t)S * n);
    e->partial = dalloc<zd>((size_t)blas_nblocks(n) * 64 * S);
    e->hdev = dalloc<zd>((size_t)4 * 64 * S);
    HIPCHK(hipHostMalloc((void**)&e->hhost, (size_t)4 * 64 * S * sizeof(zd)));
    e->rpart = dalloc<double>((size_t)2 * RESNORM_MAX_BLOCKS * S);
    e->rf_dev = dalloc<double>((size_t)S);
    HIPCHK(hipHostMalloc((void**)&e->rf_host, (size_t)S * sizeof(double)));
    e->flag_dev = dalloc<int>((size_t)2 * S);
    HIPCHK(hipHostMalloc((void**)&e->flag_host, (size_t)2 * S * sizeof(int)));
    e->id = dalloc<int>((size_t)NPH * NI * S);
    HIPCHK(hipHostMalloc((void**)&e->ih, (size_t)NPH * NI * S * sizeof(int)));
    e->cd = dalloc<double>((size_t)NPH * S);
    HIPCHK(hipHostMalloc((void**)&e->ch, (size_t)NPH * S * sizeof(double)));
    e->yd = dalloc<zd>((size_t)64 * S);
    HIPCHK(hipHostMalloc((void**)&e->yh, (size_t)64 * S * sizeof(zd)));
    e->slots.assign(S, Slot{});
    h->ensure_cap(S);
    ++h->graph_gen;  // captured graphs name the engine's buffers
  } catch (...) {
    delete e;
    throw;
  }
  return e;
}

void engine_destroy(SlotEngine* e) {
  if (!e) return;
  ++e->h->graph_gen;
  delete e;
}
int engine_capacity(const SlotEngine* e) { return e->S; }
int engine_free_slots(const SlotEngine* e) { return e->S - e->busy; }
int engine_busy(const SlotEngine* e) { return e->busy; }

int engine_admit(SlotEngine* e, const zd* b, zd* x, double tol, uint64_t tag) {
  for (int s = 0; s < e->S; ++s) {
    Slot& sl = e->slots[s];
    if (sl.state != FREE) continue;
    sl = Slot{};
    sl.state = NEW;
    sl.tag = tag;
    sl.B = b;
    sl.X = x;
    sl.tol = tol;
    sl.t0 = std::chrono::steady_clock::now();
    ++e->busy;
    return s;
  }
  return -1;
}

// ---- pre phase: bhat of new slots, norms of the residual of new and restarted slots
void engine_issue_pre(SlotEngine* e) {
  bamg_hierarchy* h = e->h;
  const size_t n = e->n;
  hipStream_t s = h->s;
  e->pre_list.clear();
  for (int q = 0; q < e->S; ++q) {
    Slot& sl = e->slots[q];
    if (sl.state == NEW) {
      launch_eo_reduce(h->f, sl.B, e->bh + (size_t)q * n, 1, s);
      launch_zero(e->flag_dev + 2 * q, 2 * sizeof(int), s);
      launch_check_finite(e->bh + (size_t)q * n, n, e->flag_dev + 2 * q, s);
      launch_fill_zero(e->xe + (size_t)q * n, n, s);
      launch_copy(e->bh + (size_t)q * n, e->rr + (size_t)q * n, n, s);
    }
    if (sl.state == NEW || sl.state == RESTART) e->pre_list.push_back(q);
  }
  const int K = (int)e->pre_list.size();
  if (K == 0) return;
  std::memcpy(e->ihost(PH_PRE, 0), e->pre_list.data(), K * sizeof(int));
  e->upload(PH_PRE, 1, K, false, 0);
  zd* out = e->hdev + (size_t)192 * e->S;
  launch_norms(e->rr, n, K, n, e->partial, out, s, e->idev(PH_PRE, 0));
  check_launch();
  HIPCHK(hipMemcpyAsync(e->hhost + (size_t)192 * e->S, out, K * sizeof(zd), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(e->flag_host, e->flag_dev, (size_t)2 * e->S * sizeof(int), hipMemcpyDeviceToHost, s));
}

void engine_finish_pre(SlotEngine* e) {
  const int K = (int)e->pre_list.size();
  if (K == 0) return;
  bamg_hierarchy* h = e->h;
  const size_t n = e->n;
  const int m = e->m;
  hipStream_t s = h->s;
  HIPCHK(hipStreamSynchronize(s));
  int ns = 0;
  int* st_slot = e->ihost(PH_START, 0);
  double* st_c = e->chost(PH_START);
  for (int k = 0; k < K; ++k) {
    const int q = e->pre_list[k];
    Slot& sl = e->slots[q];
    const double nrm = e->hhost[(size_t)192 * e->S + k].x;
    if (sl.state == NEW) {
      if (e->flag_host[2 * q]) {  // non-finite right-hand side: x is left untouched
        sl.status = BAMG_EINVAL;
        sl.state = FINISHING;
        e->finishing.push_back(q);
        continue;
      }
      sl.bnorm = std::sqrt(nrm);
      if (sl.bnorm == 0.0) sl.relres = 0.0;
    }
    if (sl.bnorm > 0.0) {
      sl.beta = std::sqrt(nrm);
      sl.relres = sl.beta / sl.bnorm;
    }
    if (sl.bnorm == 0.0 || !(sl.relres > sl.tol) || sl.it >= h->p.max_iter) {
      launch_eo_reconstruct(h->f, sl.B, e->xe + (size_t)q * n, sl.X, 1, s);
      // ||b - D x|| / ||b|| of the unreduced system, read by finish_slot after the round's sync
      launch_wilson_resnorm_packed(h->f, sl.B, sl.X, 1, e->rpart + (size_t)2 * RESNORM_MAX_BLOCKS * q,
                                   e->rf_dev + q, s);
      HIPCHK(hipMemcpyAsync(e->rf_host + q, e->rf_dev + q, sizeof(double), hipMemcpyDeviceToHost, s));
      sl.reconstructed = true;
      sl.state = FINISHING;
      e->finishing.push_back(q);
      continue;
    }
    ++sl.cycles;
    sl.j = 0;
    sl.H.assign((size_t)(m + 1) * m, C(0.0));
    sl.g.assign((size_t)m + 1, C(0.0));
    sl.sn.assign((size_t)m, C(0.0));
    sl.cs.assign((size_t)m, 0.0);
    sl.g[0] = sl.beta;
    sl.state = ARNOLDI;
    st_slot[ns] = q;
    st_c[ns] = 1.0 / sl.beta;
    ++ns;
  }
  if (ns > 0) {
    e->upload(PH_START, 1, ns, true, 0);
    const int* sl_d = e->idev(PH_START, 0);
    // V_{q,0} = r_q / beta_q
    launch_sscatter(e->rr, n, sl_d, e->V, (m + 1) * n, n, sl_d, nullptr, e->cdev(PH_START), n, ns, s);
  }
  check_launch();
}

// ---- main phase: one Arnoldi step of every slot in the Arnoldi phase
void engine_issue_main(SlotEngine* e) {
  bamg_hierarchy* h = e->h;
  const size_t n = e->n;
  const int m = e->m, S = e->S;
  e->act.clear();
  for (int q = 0; q < S; ++q)
    if (e->slots[q].state == ARNOLDI) e->act.push_back(q);
  const int A = (int)e->act.size();
  if (A == 0) return;
  int* a_slot = e->ihost(PH_MAIN, 0);
  int* a_j = e->ihost(PH_MAIN, 1);
  int* a_cnt = e->ihost(PH_MAIN, 2);
  int maxcnt = 0;
  for (int a = 0; a < A; ++a) {
    a_slot[a] = e->act[a];
    a_j[a] = e->slots[e->act[a]].j;
    a_cnt[a] = a_j[a] + 1;
    maxcnt = std::max(maxcnt, a_cnt[a]);
  }
  e->upload(PH_MAIN, 3, A, false, 0);
  const int* d_slot = e->idev(PH_MAIN, 0);
  const int* d_j = e->idev(PH_MAIN, 1);
  const int* d_cnt = e->idev(PH_MAIN, 2);
  const size_t ldsV = (size_t)(m + 1) * n, ldsZ = (size_t)m * n;
  zd* h1 = e->hdev;
  zd* h2 = e->hdev + (size_t)64 * S;
  zd* hn = e->hdev + (size_t)128 * S;
  const bool saved = h->force_mr;
  h->force_mr = true;  // the same kernels for every A: batch invariance
  // with graphs every Gram-Schmidt launch covers all m + 1 basis vectors (the
  // blocks beyond an entry's count exit), so one graph serves each A
  const int mc = h->p.graphs ? m + 1 : maxcnt;
  try {
    h->run_graph((1ull << 40) | (uint64_t)A, [&] {
      hipStream_t sc = h->s;
      launch_sgather(e->V, ldsV, n, d_slot, d_j, e->cur, n, A, sc);
      h->precondition(e->cur, e->zc, A);
      launch_sscatter(e->zc, n, nullptr, e->Z, ldsZ, n, d_slot, d_j, nullptr, n, A, sc);
      h->apply(0, e->zc, e->w, nullptr, A);
      launch_smultidot(e->V, ldsV, n, d_slot, d_cnt, mc, e->w, n, A, e->partial, h1, sc);
      launch_smultiaxpy(e->V, ldsV, n, d_slot, d_cnt, h1, -1.0, e->w, n, A, sc);
      launch_smultidot(e->V, ldsV, n, d_slot, d_cnt, mc, e->w, n, A, e->partial, h2, sc);
      launch_smultiaxpy(e->V, ldsV, n, d_slot, d_cnt, h2, -1.0, e->w, n, A, sc);
      launch_norms(e->w, n, A, n, e->partial, hn, sc);
      check_launch();
      HIPCHK(hipMemcpyAsync(e->hhost, e->hdev, ((size_t)128 * S + A) * sizeof(zd), hipMemcpyDeviceToHost, sc));
    });
  } catch (...) {
    h->force_mr = saved;
    throw;
  }
  h->force_mr = saved;
}

void engine_finish_main(SlotEngine* e, std::vector<SlotDone>& done) {
  bamg_hierarchy* h = e->h;
  const size_t n = e->n;
  const int m = e->m, S = e->S;
  hipStream_t s = h->s;
  const int A = (int)e->act.size();
  if (A == 0 && e->finishing.empty()) return;
  HIPCHK(hipStreamSynchronize(s));
  for (int q : e->finishing) e->finish_slot(q, done);
  e->finishing.clear();
  if (A == 0) return;
  const zd* hh = e->hhost;
  int nc = 0, ne = 0;
  int* c_slot = e->ihost(PH_POST, 0);
  int* c_j = e->ihost(PH_POST, 1);
  int* c_src = e->ihost(PH_POST, 2);
  int* e_slot = e->ihost(PH_POST, 3);
  int* e_cnt = e->ihost(PH_POST, 4);
  double* c_c = e->chost(PH_POST);
  std::vector<int> failed;
  for (int a = 0; a < A; ++a) {
    const int q = e->act[a];
    Slot& sl = e->slots[q];
    const int j = sl.j;
    C* Hr = sl.H.data();
    C* gr = sl.g.data();
    for (int k = 0; k <= j; ++k)
      Hr[(size_t)k * m + j] = C(hh[a * 64 + k].x, hh[a * 64 + k].y) +
                              C(hh[(size_t)64 * S + a * 64 + k].x, hh[(size_t)64 * S + a * 64 + k].y);
    const double hnv = std::sqrt(hh[(size_t)128 * S + a].x);
    if (!std::isfinite(hnv)) {
      sl.status = BAMG_EDEVICE;
      failed.push_back(q);
      continue;
    }
    // previous rotations, then the new one (eliminates h_{j+1,j})
    for (int k = 0; k < j; ++k) {
      const C x0 = Hr[(size_t)k * m + j], x1 = Hr[(size_t)(k + 1) * m + j];
      Hr[(size_t)k * m + j] = sl.cs[k] * x0 + sl.sn[k] * x1;
      Hr[(size_t)(k + 1) * m + j] = -std::conj(sl.sn[k]) * x0 + sl.cs[k] * x1;
    }
    const C x0 = Hr[(size_t)j * m + j];
    const double ax = std::abs(x0);
    double c;
    C sv;
    if (hnv == 0.0) { c = 1.0; sv = 0.0; }
    else if (ax == 0.0) { c = 0.0; sv = 1.0; }
    else {
      const double t = std::sqrt(ax * ax + hnv * hnv);
      c = ax / t;
      sv = (x0 / ax) * (hnv / t);
    }
    sl.cs[j] = c;
    sl.sn[j] = sv;
    Hr[(size_t)j * m + j] = c * x0 + sv * hnv;
    gr[j + 1] = -std::conj(sv) * gr[j];
    gr[j] = c * gr[j];
    ++sl.it;
    const bool end = std::abs(gr[j + 1]) <= sl.tol * sl.bnorm || sl.it >= h->p.max_iter || hnv == 0.0 || j + 1 == m;
    if (!end) {
      c_slot[nc] = q;
      c_j[nc] = j + 1;
      c_src[nc] = a;
      c_c[nc] = 1.0 / hnv;
      ++nc;
      sl.j = j + 1;
      continue;
    }
    // y = H^{-1} g on the leading jend x jend upper triangle
    const int jend = j + 1;
    std::vector<C> y(jend);
    for (int i = jend - 1; i >= 0; --i) {
      C sum = gr[i];
      for (int k = i + 1; k < jend; ++k) sum -= Hr[(size_t)i * m + k] * y[k];
      y[i] = sum / Hr[(size_t)i * m + i];
    }
    zd* yrow = e->yh + (size_t)ne * 64;
    for (int k = 0; k < 64; ++k) yrow[k] = zd{0, 0};
    for (int k = 0; k < jend; ++k) yrow[k] = zd{y[k].real(), y[k].imag()};
    e_slot[ne] = q;
    e_cnt[ne] = jend;
    ++ne;
    sl.state = RESTART;
  }
  const int K = std::max(nc, ne);
  if (K > 0) {
    e->upload(PH_POST, 5, K, nc > 0, ne);
    const size_t ldsV = (size_t)(m + 1) * n, ldsZ = (size_t)m * n;
    // continuing slots: V_{q,j+1} = w_a / h_{j+1,j}
    launch_sscatter(e->w, n, e->idev(PH_POST, 2), e->V, ldsV, n, e->idev(PH_POST, 0), e->idev(PH_POST, 1),
                    e->cdev(PH_POST), n, nc, s);
    // slots at the end of a restart cycle: x_e += Z y, then r = bhat - Dhat x_e
    if (ne > 0) {
      const int* d_es = e->idev(PH_POST, 3);
      launch_slincomb(e->Z, ldsZ, n, d_es, e->idev(PH_POST, 4), e->yd, e->xe, n, ne, s);
      launch_sgather(e->xe, n, 0, d_es, nullptr, e->cur, n, ne, s);
      launch_sgather(e->bh, n, 0, d_es, nullptr, e->zc, n, ne, s);
      h->apply(0, e->cur, e->w, e->zc, ne);
      launch_sscatter(e->w, n, nullptr, e->rr, n, 0, d_es, nullptr, nullptr, n, ne, s);
    }
    check_launch();
  }
  for (int q : failed) e->finish_slot(q, done);
}

}  // namespace bamg
