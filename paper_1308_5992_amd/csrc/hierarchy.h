// Internal: the hierarchy of levels (operators, interpolation, smoother data,
// work vectors) and the host-side orchestration of its kernels, shared by the
// C ABI (bamg_host.cpp), the slot-based batched Krylov engine (engine.cpp)
// and the serving scheduler (server.cpp).  Not part of the public interface.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <complex>
#include <map>
#include <string>
#include <vector>

#include "../../include/bamg.h"
#include "bamg_internal.h"

namespace bamg {

#define HIPCHK(expr)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      throw HipFail(std::string(#expr) + ": " + hipGetErrorString(e_));                    \
  } while (0)

struct HipFail {
  std::string msg;
  explicit HipFail(std::string m) : msg(std::move(m)) {}
};
struct BadArg {
  std::string msg;
  explicit BadArg(std::string m) : msg(std::move(m)) {}
};

inline void check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw HipFail(std::string("kernel launch: ") + hipGetErrorString(e));
}

template <typename T>
inline T* dalloc(size_t count) {
  void* p = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc(&p, count * sizeof(T));
  if (e != hipSuccess) throw HipFail(std::string("hipMalloc: ") + hipGetErrorString(e));
  return (T*)p;
}

inline void dfree(void* p) {
  if (p) (void)hipFree(p);
}

inline int floor_mod(int a, int n) { return ((a % n) + n) % n; }

// right-hand sides from which the smoothers use their multi-RHS kernels
constexpr int MR_MIN = 4;

// ---- multicolour orderings (Sec. 3.1 leaves the colouring open) -------------
// fine even site (x, y): 4 * (((x+y)/2) mod 4) + (((x-y)/2) mod 4); 16 colours
inline int fine_colour_of(int x, int y) { return 4 * floor_mod((x + y) / 2, 4) + floor_mod((x - y) / 2, 4); }
// coarse site (ax, ay): 8 colours (ax - 3 ay) mod 8 if both extents are
// multiples of 8, else 16 colours 4 (ay mod 4) + (ax mod 4) if multiples of 4,
// else one site per colour
inline int coarse_ncol(int ex, int ey) {
  if (ex % 8 == 0 && ey % 8 == 0) return 8;
  if (ex % 4 == 0 && ey % 4 == 0) return 16;
  return ex * ey;
}

struct SlotEngine;
void engine_destroy(SlotEngine* e);

}  // namespace bamg

using namespace bamg;

struct Level {
  int ex = 0, ey = 0, dps = 0;
  size_t n = 0;                 // dofs
  zd* D = nullptr;              // coarse block stencil (levels >= 1)
  zd* Kinv = nullptr;           // smoother data (non-coarsest coarse levels)
  zd* Ainv = nullptr;           // inverse of the coarsest operator
  int ncol = 0, cmode = 0, per_colour = 0;  // smoother colours, colouring mode, sites per colour
  zd* P = nullptr;              // interpolation from level l+1 (non-coarsest levels)
  int prow = 0;                 // rows of P_{a,s}
  zd *x = nullptr, *b = nullptr, *r = nullptr;  // work vectors, cap right-hand sides
  zd* tv = nullptr;             // test vectors on this level [k][n]
  // mixed-precision cycle: FP32 interpolation and smoother data, operator in
  // the storage type of the hierarchy (FP32, FP16 or BF16), FP32 work vectors
  zf* P32 = nullptr;
  void* Dst = nullptr;
  zf* Kinv32 = nullptr;
  zf *x32 = nullptr, *b32 = nullptr, *r32 = nullptr;
  Coarse coarse() const {
    Coarse c;
    c.ex = ex; c.ey = ey; c.D = D; c.Kinv = Kinv;
    return c;
  }
};

struct bamg_hierarchy {
  bamg_params p{};
  double m = 0;
  hipStream_t s = nullptr;
  Fine f;
  zd *Ue = nullptr, *Uo = nullptr, *Bst = nullptr;
  FineT<float> f32;
  zf *Ue32 = nullptr, *Uo32 = nullptr, *Bst32 = nullptr;
  std::vector<Level> lv;
  int cap = 0;  // right-hand sides the work vectors hold
  // batched path: multi-RHS kernels for every batch size, so that a right-hand
  // side's arithmetic does not depend on how many others share the batch
  bool force_mr = false;
  zd* mmwork = nullptr;  // split-K partials of the coarsest product, cap right-hand sides
  // coarsest inversion scratch
  zd* gjcol = nullptr;
  int* gjperm = nullptr;
  int* dflag = nullptr;   // device flag
  int* hflag = nullptr;   // pinned host mirror
  // Krylov workspace for kcap right-hand sides (basis layout [j][r][n])
  int kdim = 0, kcap = 0;
  zd *V = nullptr, *Z = nullptr, *w = nullptr, *bh = nullptr, *xe = nullptr, *rr = nullptr;
  zd *partial = nullptr, *hdev = nullptr;  // reduction partials; [3][kcap][64] results
  zd* hhost = nullptr;                     // pinned mirror of hdev
  double *scal_dev = nullptr, *scal_host = nullptr;  // per right-hand side scale factors
  zd *ycoef_dev = nullptr, *ycoef_host = nullptr;    // per right-hand side update coefficients
  zd* tvsave = nullptr; // level-0 test vectors after the last setup pass
  SlotEngine* engine = nullptr;  // batched solves (slot engine, created on first use)
  // captured launch sequences (p.graphs): one executable graph per key, valid
  // while the buffers they name stay allocated (graph_gen counts reallocations)
  std::map<uint64_t, hipGraphExec_t> graphs;
  uint64_t graph_gen = 0, graphs_gen = 0;
  hipStream_t cap_stream = nullptr;

  void drop_graphs() {
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    graphs.clear();
  }
  // run issue() (launches on `s`) directly, or as the replay of its captured graph
  template <typename F>
  void run_graph(uint64_t key, F&& issue) {
    if (!p.graphs) {
      issue();
      return;
    }
    if (graphs_gen != graph_gen) {
      drop_graphs();
      graphs_gen = graph_gen;
    }
    auto it = graphs.find(key);
    if (it == graphs.end()) {
      if (!cap_stream) HIPCHK(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
      hipStream_t saved = s;
      s = cap_stream;
      HIPCHK(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeRelaxed));
      hipGraph_t g = nullptr;
      try {
        issue();
      } catch (...) {
        (void)hipStreamEndCapture(cap_stream, &g);
        if (g) (void)hipGraphDestroy(g);
        s = saved;
        throw;
      }
      s = saved;
      HIPCHK(hipStreamEndCapture(cap_stream, &g));
      hipGraphExec_t ex = nullptr;
      const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) throw HipFail(std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
      it = graphs.emplace(key, ex).first;
    }
    HIPCHK(hipGraphLaunch(it->second, s));
  }

  void free_krylov() {
    dfree(V); dfree(Z); dfree(w); dfree(bh); dfree(xe); dfree(rr); dfree(partial); dfree(hdev);
    dfree(scal_dev); dfree(ycoef_dev);
    if (hhost) (void)hipHostFree(hhost);
    if (scal_host) (void)hipHostFree(scal_host);
    if (ycoef_host) (void)hipHostFree(ycoef_host);
    V = Z = w = bh = xe = rr = partial = hdev = hhost = ycoef_dev = ycoef_host = nullptr;
    scal_dev = scal_host = nullptr;
    kcap = 0;
  }
  // reduction scratch for at least R right-hand sides (always), Krylov bases if `bases`
  void ensure_krylov(int R, bool bases) {
    const size_t n0 = lv[0].n;
    if (R > kcap || (bases && !V)) {
      ++graph_gen;
      const int cap2 = std::max(R, kcap);
      const bool had_bases = V != nullptr || bases;
      free_krylov();
      kcap = cap2;
      partial = dalloc<zd>((size_t)blas_nblocks(n0) * 64 * kcap);
      hdev = dalloc<zd>((size_t)3 * 64 * kcap);
      HIPCHK(hipHostMalloc((void**)&hhost, (size_t)3 * 64 * kcap * sizeof(zd)));
      scal_dev = dalloc<double>(kcap);
      HIPCHK(hipHostMalloc((void**)&scal_host, (size_t)kcap * sizeof(double)));
      ycoef_dev = dalloc<zd>((size_t)64 * kcap);
      HIPCHK(hipHostMalloc((void**)&ycoef_host, (size_t)64 * kcap * sizeof(zd)));
      if (had_bases) {
        V = dalloc<zd>(n0 * (kdim + 1) * kcap);
        Z = dalloc<zd>(n0 * kdim * kcap);
        w = dalloc<zd>(n0 * kcap);
        bh = dalloc<zd>(n0 * kcap);
        xe = dalloc<zd>(n0 * kcap);
        rr = dalloc<zd>(n0 * kcap);
      }
    }
  }

  ~bamg_hierarchy() {
    for (auto& L : lv) {
      dfree(L.D); dfree(L.Kinv); dfree(L.Ainv); dfree(L.P);
      dfree(L.x); dfree(L.b); dfree(L.r); dfree(L.tv);
      dfree(L.P32); dfree(L.Dst); dfree(L.Kinv32); dfree(L.x32); dfree(L.b32); dfree(L.r32);
    }
    dfree(mmwork);
    dfree(Ue); dfree(Uo); dfree(Ue32); dfree(Uo32); dfree(Bst); dfree(Bst32); dfree(gjcol); dfree(gjperm); dfree(dflag);
    if (hflag) (void)hipHostFree(hflag);
    free_krylov();
    dfree(tvsave);
    if (engine) engine_destroy(engine);
    drop_graphs();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
  }

  int L() const { return (int)lv.size(); }
  bool coarsest(int l) const { return l == L() - 1; }

  bool mixed() const { return p.precision != BAMG_FP64; }

  void ensure_cap(int nrhs) {
    if (nrhs <= cap) return;
    ++graph_gen;
    dfree(mmwork);
    mmwork = nullptr;
    if (L() > 1) mmwork = dalloc<zd>(dense_mm_workspace((int)lv.back().n, nrhs));
    for (auto& Lv : lv) {
      dfree(Lv.x); dfree(Lv.b); dfree(Lv.r);
      dfree(Lv.x32); dfree(Lv.b32); dfree(Lv.r32);
      Lv.x32 = Lv.b32 = Lv.r32 = nullptr;
      Lv.x = dalloc<zd>(Lv.n * nrhs);
      Lv.b = dalloc<zd>(Lv.n * nrhs);
      Lv.r = dalloc<zd>(Lv.n * nrhs);
      if (mixed()) {
        Lv.x32 = dalloc<zf>(Lv.n * nrhs);
        Lv.b32 = dalloc<zf>(Lv.n * nrhs);
        Lv.r32 = dalloc<zf>(Lv.n * nrhs);
      }
    }
    cap = nrhs;
  }

  // ---------------------------------------------------------------- level ops
  void apply(int l, const zd* x, zd* y, const zd* b, int nrhs) {
    if (l == 0) launch_dhat(f, x, y, b, nrhs, s);
    else launch_coarse_apply(lv[l].coarse(), x, y, b, nrhs, s);
    check_launch();
  }
  void sweep(int l, zd* x, const zd* b, int nrhs) {
    Level& Lv = lv[l];
    for (int c = 0; c < Lv.ncol; ++c) {
      if (l == 0) launch_kaczmarz_fine(f, c, Lv.per_colour, x, b, nrhs, s);
      else launch_kaczmarz_coarse(Lv.coarse(), c, Lv.cmode, Lv.per_colour, x, b, nrhs, s);
    }
    check_launch();
  }
  void restrict_(int l, const zd* r, zd* rc, int nrhs) {
    if (l == 0) launch_restrict_fine(f, lv[0].P, r, rc, nrhs, s);
    else launch_restrict_coarse(lv[l].ex, lv[l].ey, lv[l].P, r, rc, nrhs, s);
    check_launch();
  }
  void prolong(int l, const zd* xc, zd* x, int nrhs) {
    if (l == 0) launch_prolong_fine(f, lv[0].P, xc, x, nrhs, s);
    else launch_prolong_coarse(lv[l].ex, lv[l].ey, lv[l].P, xc, x, nrhs, s);
    check_launch();
  }
  void coarsest_solve(const zd* b, zd* x, int nrhs) {
    Level& Lv = lv.back();
    if (nrhs > cap) throw HipFail("coarsest solve: more right-hand sides than the workspace holds");
    launch_dense_mv(Lv.Ainv, (int)Lv.n, b, x, nrhs, force_mr, mmwork, s);
    check_launch();
  }

  // multigrid cycle on level l for A_l x = b, x holds the initial guess
  // (pre-smoothing, residual, restriction, coarse correction, prolongation,
  // post-smoothing; Sec. 1 two-grid scheme applied recursively, Sec. 4)
  void cycle(int l, const zd* b, zd* x, int nrhs) {
    if (L() == 1) {  // one level: the cycle reduces to its smoothing sweeps
      for (int i = 0; i < p.pre + p.post; ++i) sweep(0, x, b, nrhs);
      return;
    }
    if (coarsest(l)) {
      coarsest_solve(b, x, nrhs);
      return;
    }
    Level& Lv = lv[l];
    Level& C = lv[l + 1];
    for (int i = 0; i < p.pre; ++i) sweep(l, x, b, nrhs);
    apply(l, x, Lv.r, b, nrhs);  // r = b - A x
    restrict_(l, Lv.r, C.b, nrhs);
    launch_fill_zero(C.x, C.n * nrhs, s);
    const int gamma = (p.cycle == BAMG_CYCLE_W) ? 2 : 1;
    for (int g = 0; g < gamma; ++g) {
      cycle(l + 1, C.b, C.x, nrhs);
      if (coarsest(l + 1)) break;
    }
    prolong(l, C.x, x, nrhs);
    for (int i = 0; i < p.post; ++i) sweep(l, x, b, nrhs);
  }

  // ------------------------------------------------ mixed-precision cycle
  // The preconditioner of the mixed modes: the same cycle in FP32 with the
  // coarse operators read from their reduced-precision copies and the
  // coarsest level solved with the FP64 inverse (FP64 in, FP64 out).
  template <typename S>
  CoarseT<float, S> coarse32(int l) const {
    CoarseT<float, S> c;
    c.ex = lv[l].ex; c.ey = lv[l].ey; c.D = (const S*)lv[l].Dst; c.Kinv = lv[l].Kinv32;
    return c;
  }
  template <typename S>
  void apply32(int l, const zf* x, zf* y, const zf* b, int nrhs) {
    if (l == 0) launch_dhat(f32, x, y, b, nrhs, s);
    else launch_coarse_apply(coarse32<S>(l), x, y, b, nrhs, s);
  }
  template <typename S>
  void sweep32(int l, zf* x, const zf* b, int nrhs) {
    Level& Lv = lv[l];
    const bool mr = force_mr || nrhs >= MR_MIN;
    for (int c = 0; c < Lv.ncol; ++c) {
      if (l == 0) {
        launch_kaczmarz_fine(f32, c, Lv.per_colour, x, b, nrhs, s);
      } else {
        if (mr) launch_kaczmarz_coarse_mfma(coarse32<S>(l), c, Lv.cmode, Lv.per_colour, x, b, nrhs, s);
        else launch_kaczmarz_coarse(coarse32<S>(l), c, Lv.cmode, Lv.per_colour, x, b, nrhs, s);
      }
    }
  }
  template <typename S>
  void cycle32(int l, const zf* b, zf* x, int nrhs) {
    if (L() == 1) {
      for (int i = 0; i < p.pre + p.post; ++i) sweep32<S>(0, x, b, nrhs);
      check_launch();
      return;
    }
    if (coarsest(l)) {
      Level& C = lv[l];
      if (nrhs > cap) throw HipFail("coarsest solve: more right-hand sides than the workspace holds");
      launch_convert(b, C.b, C.n * nrhs, s);
      launch_dense_mv(C.Ainv, (int)C.n, C.b, C.x, nrhs, force_mr, mmwork, s);
      launch_convert(C.x, x, C.n * nrhs, s);
      check_launch();
      return;
    }
    Level& Lv = lv[l];
    Level& C = lv[l + 1];
    for (int i = 0; i < p.pre; ++i) sweep32<S>(l, x, b, nrhs);
    apply32<S>(l, x, Lv.r32, b, nrhs);
    if (l == 0) launch_restrict_fine(f32, Lv.P32, Lv.r32, C.b32, nrhs, s);
    else launch_restrict_coarse(Lv.ex, Lv.ey, Lv.P32, Lv.r32, C.b32, nrhs, s);
    launch_zero(C.x32, C.n * nrhs * sizeof(zf), s);
    const int gamma = (p.cycle == BAMG_CYCLE_W) ? 2 : 1;
    for (int g = 0; g < gamma; ++g) {
      cycle32<S>(l + 1, C.b32, C.x32, nrhs);
      if (coarsest(l + 1)) break;
    }
    if (l == 0) launch_prolong_fine(f32, Lv.P32, C.x32, x, nrhs, s);
    else launch_prolong_coarse(Lv.ex, Lv.ey, Lv.P32, C.x32, x, nrhs, s);
    for (int i = 0; i < p.post; ++i) sweep32<S>(l, x, b, nrhs);
    check_launch();
  }
  // z = M v for nrhs FP64 level-0 vectors through the FP32 cycle
  void precondition_mixed(const zd* v, zd* z, int nrhs) {
    Level& L0 = lv[0];
    launch_convert(v, L0.b32, L0.n * nrhs, s);
    launch_zero(L0.x32, L0.n * nrhs * sizeof(zf), s);
    switch (p.precision) {
      case BAMG_MIXED_FP16: cycle32<hcx>(0, L0.b32, L0.x32, nrhs); break;
      case BAMG_MIXED_BF16: cycle32<bcx>(0, L0.b32, L0.x32, nrhs); break;
      default: cycle32<zf>(0, L0.b32, L0.x32, nrhs); break;
    }
    launch_convert(L0.x32, z, L0.n * nrhs, s);
    check_launch();
  }
  // z = M v in the hierarchy's precision
  void precondition(const zd* v, zd* z, int nrhs) {
    if (mixed()) {
      precondition_mixed(v, z, nrhs);
    } else {
      launch_fill_zero(z, lv[0].n * nrhs, s);
      cycle(0, v, z, nrhs);
    }
  }
  template <typename S>
  void store_op(int l) {
    Level& Lv = lv[l];
    const size_t ne = (size_t)Lv.ex * Lv.ey * NOFF * 256;
    if (!Lv.Dst) Lv.Dst = dalloc<S>(ne);
    launch_convert(Lv.D, (S*)Lv.Dst, ne, s);
    if (!coarsest(l)) {
      if (!Lv.Kinv32) Lv.Kinv32 = dalloc<zf>((size_t)Lv.ex * Lv.ey * 256);
      launch_kaczmarz_prep(coarse32<S>(l), Lv.Kinv32, s);
    }
  }
  // reduced-precision copies of the solve-phase data (after setup / import)
  void refresh_mixed() {
    if (!mixed()) return;
    const size_t nl = (size_t)f.N * f.N;
    if (!Ue32) {
      Ue32 = dalloc<zf>(nl);
      Uo32 = dalloc<zf>(nl);
    }
    launch_convert(Ue, Ue32, nl, s);
    launch_convert(Uo, Uo32, nl, s);
    f32.N = f.N; f32.NH = f.NH; f32.c = f.c; f32.kappa = f.kappa; f32.kappa2 = f.kappa2;
    f32.Ue = Ue32; f32.Uo = Uo32;
    if (!Bst32) Bst32 = dalloc<zf>(nl / 2 * 36);
    launch_slot_blocks(f32, Bst32, s);
    f32.Bst = Bst32;
    for (int l = 0; l < L(); ++l) {
      Level& Lv = lv[l];
      if (Lv.P) {
        if (!Lv.P32) Lv.P32 = dalloc<zf>(Lv.n * 8);
        launch_convert(Lv.P, Lv.P32, Lv.n * 8, s);
      }
      if (l >= 1 && !(coarsest(l) && L() > 1)) {
        switch (p.precision) {
          case BAMG_MIXED_FP16: store_op<hcx>(l); break;
          case BAMG_MIXED_BF16: store_op<bcx>(l); break;
          default: store_op<zf>(l); break;
        }
      }
    }
    check_launch();
    HIPCHK(hipStreamSynchronize(s));
  }

  // ---------------------------------------------------------------- setup
  // colour classes of the smoother (the kernels enumerate the sites of a
  // colour arithmetically)
  void build_colours(int l) {
    Level& Lv = lv[l];
    if (l == 0) {
      Lv.ncol = 16;
      Lv.cmode = 0;
      Lv.per_colour = f.N * f.N / 32;
    } else {
      Lv.ncol = coarse_ncol(Lv.ex, Lv.ey);
      Lv.cmode = Lv.ncol == 8 ? 8 : (Lv.ncol == 16 ? 16 : 1);
      Lv.per_colour = Lv.ex * Lv.ey / (Lv.cmode == 1 ? Lv.ex * Lv.ey : Lv.cmode);
    }
  }

  // D_{l+1} from P_l, then its smoother data or (coarsest) its inverse
  void build_next(int l) {
    Level& C = lv[l + 1];
    if (l == 0) launch_galerkin_fine(f, lv[0].P, C.D, s);
    else launch_galerkin_coarse(lv[l].coarse(), lv[l].P, C.D, s);
    check_launch();
    if (!coarsest(l + 1)) {
      launch_kaczmarz_prep(C.coarse(), C.Kinv, s);
      check_launch();
    } else {
      invert_coarsest();
    }
  }

  void invert_coarsest() {
    Level& C = lv.back();
    const int n = (int)C.n;
    launch_densify(C.coarse(), C.Ainv, s);
    HIPCHK(hipMemsetAsync(dflag, 0, sizeof(int), s));
    launch_gj_invert(C.Ainv, n, gjcol, gjperm, dflag, s);
    launch_gj_unpermute(C.Ainv, n, gjperm, s);
    check_launch();
    HIPCHK(hipMemcpyAsync(hflag, dflag, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (*hflag) throw BadArg("singular coarsest operator");
  }

  void fit(int l, const zd* V) {
    if (l == 0) launch_fit_fine(f, V, p.n_tv, lv[0].P, s);
    else launch_fit_coarse(lv[l].coarse(), V, p.n_tv, lv[l].P, s);
    check_launch();
  }

  // relax -> normalise -> fit -> Galerkin -> restrict, level by level, from
  // the level-0 test vectors in lv[0].tv
  void setup_pass() {
    const int k = p.n_tv;
    for (int l = 0; l + 1 < L(); ++l) {
      Level& Lv = lv[l];
      for (int i = 0; i < p.setup_sweeps; ++i) sweep(l, Lv.tv, nullptr, k);
      launch_norms(Lv.tv, Lv.n, k, Lv.n, partial, hdev, s);
      launch_normalize(Lv.tv, Lv.n, k, Lv.n, hdev, s);
      check_launch();
      if (l == 0) launch_copy(Lv.tv, tvsave, Lv.n * k, s);
      fit(l, Lv.tv);
      build_next(l);
      restrict_(l, Lv.tv, lv[l + 1].tv, k);
    }
    HIPCHK(hipStreamSynchronize(s));
  }
};

namespace bamg {

// ---- slot-based Krylov engine (engine.cpp) -----------------------------------
// FGMRES(restart) in FP64 for up to `slots` right-hand sides of one hierarchy
// that enter and leave independently (continuous batching).  All right-hand
// sides in the Arnoldi phase advance together, one iteration per round, with
// the batch-invariant multi-RHS kernels; a right-hand side's arithmetic is
// the same whatever the other slots hold, so its result is bitwise
// independent of when it entered and of what it shared the device with.
struct SlotEngine;
struct SlotDone {
  uint64_t tag;
  int status;  // BAMG_OK, BAMG_NOT_CONVERGED or BAMG_EDEVICE
  bamg_solve_info info;
};
SlotEngine* engine_create(bamg_hierarchy* h, int slots);  // throws HipFail
void engine_destroy(SlotEngine* e);
size_t engine_slot_bytes(size_t n0, int restart, int slots);  // device bytes of the slots
int engine_capacity(const SlotEngine* e);
int engine_free_slots(const SlotEngine* e);
int engine_busy(const SlotEngine* e);  // slots in use
// reserve a slot for b (full lattice, device) -> x; the work starts at the next round
int engine_admit(SlotEngine* e, const zd* b, zd* x, double tol, uint64_t tag);
// one round, split so that several engines on different streams overlap:
// pre (norms of new and restarted slots), main (one Arnoldi step of every
// active slot); each issue_* only launches, each finish_* synchronises the
// engine's stream and does the host algebra.  Finished right-hand sides are
// appended to `done` by finish_main (their x is complete at that point).
void engine_issue_pre(SlotEngine* e);
void engine_finish_pre(SlotEngine* e);
void engine_issue_main(SlotEngine* e);
void engine_finish_main(SlotEngine* e, std::vector<SlotDone>& done);

// device bytes that holding `slots` right-hand sides adds to a hierarchy's
// level work vectors (bamg_footprint_bytes counts one)
size_t hierarchy_slot_extra_bytes(const bamg_params* p, int slots);
// record `msg` as this thread's bamg_last_error() text and return code
int api_fail(int code, const std::string& msg);

}  // namespace bamg
