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
// from this many right-hand sides the level-0 smoothing sweeps run on
// right-hand-side-interleaved copies of x and b (launch_smooth_fine_il),
// below IL_BLOCKED only where the streaming blocked sweep does not apply
constexpr int IL_MIN = 16;
constexpr int IL_BLOCKED = 32;
// offset (entries) of the second set of single-RHS reduction results in
// hdev / hhost: past the first set's [3][64] and the solve's own slots after it
constexpr size_t HSET1 = 192;

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
  zd* Ap = nullptr;             // its blocks on and above the block diagonal (single-RHS product)
  int* Ablk = nullptr;          // (I, J) of each packed block
  zd* Apart = nullptr;          // partial products of the packed form, 2 right-hand sides
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
  zf* Ainv32 = nullptr;         // FP32 copy of the coarsest inverse
  zf* Ap32 = nullptr;           // FP32 copy of its packed blocks (single-RHS product)
  zf *x32 = nullptr, *b32 = nullptr, *r32 = nullptr;
  // K-cycle visits of this level (1 <= l <= L-2): z1, w1, r1, z2, w2 for cap
  // right-hand sides each, in FP64 and (mixed modes) FP32; 4 coefficients per
  // right-hand side
  zd* kw = nullptr;
  zf* kw32 = nullptr;
  zd* kcoef = nullptr;
  // second copy of x for the fused colour-pair passes (non-coarsest coarse
  // levels), cap right-hand sides, FP64 and (mixed modes) FP32
  zd* xs = nullptr;
  zf* xs32 = nullptr;
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
  zd *Ue = nullptr, *Uo = nullptr, *Bst = nullptr, *Gst = nullptr;
  FineT<float> f32;
  zf *Ue32 = nullptr, *Uo32 = nullptr, *Bst32 = nullptr, *Gst32 = nullptr;
  std::vector<Level> lv;
  int cap = 0;  // right-hand sides the work vectors hold
  // batched path: multi-RHS kernels for every batch size, so that a right-hand
  // side's arithmetic does not depend on how many others share the batch
  bool force_mr = false;
  zd* mmwork = nullptr;  // split-K partials of the coarsest product, cap right-hand sides
  zd* kpart = nullptr;   // reduction partials of the K-cycle visits, cap right-hand sides
  // level-0 right-hand-side-interleaved x and b for the smoothing sweeps (cap >= IL_MIN)
  zd *xil = nullptr, *bil = nullptr;
  zf *xil32 = nullptr, *bil32 = nullptr;
  // level-0 second copy of x for the sweeps blocked in LDS (they read one
  // copy and write the other), cap right-hand sides
  zd* xsw = nullptr;
  zf* xsw32 = nullptr;
  // coarsest inversion scratch
  zd* gjcol = nullptr;
  int* gjperm = nullptr;
  int* dflag = nullptr;   // device flag
  int* hflag = nullptr;   // pinned host mirror
  // Krylov workspace for kcap right-hand sides (basis layout [j][r][n])
  int kdim = 0, kcap = 0;
  zd *V = nullptr, *Z = nullptr, *w = nullptr, *bh = nullptr, *xe = nullptr, *rr = nullptr;
  // reduction partials; results [3][kcap][64], then for a single right-hand
  // side a second set of [3][64] (FGMRES iterations of odd index, so that one
  // iteration can run while the host reads the results of the one before)
  zd *partial = nullptr, *hdev = nullptr;
  zd* hhost = nullptr;                     // pinned mirror of hdev
  hipEvent_t ev_iter = nullptr;            // end of an FGMRES iteration (look-ahead)
  double *scal_dev = nullptr, *scal_host = nullptr;  // per right-hand side scale factors
  zd *ycoef_dev = nullptr, *ycoef_host = nullptr;    // per right-hand side update coefficients
  zd* tvsave = nullptr; // level-0 test vectors after the last setup pass
  SlotEngine* engine = nullptr;  // batched solves (slot engine, created on first use)
  // bootstrap eigensolver state (setup_mode 1, 2): per level the test vectors
  // are [V^r (n_tv) | V^e (ke)] in Level::tv; Ritz values on the device
  int ke = 0;
  bool have_e = false;
  double *lam_dev = nullptr, *lam_host = nullptr;
  zd *eigX = nullptr, *eigY = nullptr, *eigT = nullptr, *eigR = nullptr, *eigC = nullptr, *eigW = nullptr;
  zd* eigH = nullptr;  // pinned host p x p
  std::vector<double> lam_final;  // Ritz values at the end of the bootstrap setup
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
      partial = dalloc<zd>((size_t)blas_nblocks_fine(n0) * 64 * kcap);  // the finer of the two block counts
      hdev = dalloc<zd>((size_t)3 * 64 * kcap + HSET1);
      // coherent: the Gram-Schmidt reductions write their results here directly
      HIPCHK(hipHostMalloc((void**)&hhost, ((size_t)3 * 64 * kcap + HSET1) * sizeof(zd), hipHostMallocCoherent));
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
      dfree(L.D); dfree(L.Kinv); dfree(L.Ainv); dfree(L.Ap); dfree(L.Ablk); dfree(L.Apart); dfree(L.P);
      dfree(L.x); dfree(L.b); dfree(L.r); dfree(L.tv);
      dfree(L.P32); dfree(L.Dst); dfree(L.Kinv32); dfree(L.Ainv32); dfree(L.Ap32); dfree(L.x32); dfree(L.b32); dfree(L.r32);
      dfree(L.kw); dfree(L.kw32); dfree(L.kcoef); dfree(L.xs); dfree(L.xs32);
    }
    dfree(mmwork);
    dfree(kpart);
    dfree(xil); dfree(bil); dfree(xil32); dfree(bil32); dfree(xsw); dfree(xsw32);
    dfree(Ue); dfree(Uo); dfree(Ue32); dfree(Uo32); dfree(Bst); dfree(Bst32); dfree(Gst); dfree(Gst32); dfree(gjcol); dfree(gjperm); dfree(dflag);
    if (hflag) (void)hipHostFree(hflag);
    free_krylov();
    dfree(tvsave);
    if (engine) engine_destroy(engine);
    dfree(lam_dev); dfree(eigX); dfree(eigY); dfree(eigT); dfree(eigR); dfree(eigC); dfree(eigW); dfree(eigmm);
    if (lam_host) (void)hipHostFree(lam_host);
    if (eigH) (void)hipHostFree(eigH);
    drop_graphs();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (ev_iter) (void)hipEventDestroy(ev_iter);
  }

  int L() const { return (int)lv.size(); }
  bool coarsest(int l) const { return l == L() - 1; }

  bool mixed() const { return p.precision != BAMG_FP64; }
  // level l takes Krylov-accelerated visits (K-cycle, l not the finest nor the coarsest)
  bool kvisited(int l) const { return p.cycle == BAMG_CYCLE_K && l >= 1 && l + 1 < L(); }
  bool c32() const { return mixed() && p.coarsest_fp32; }

  void ensure_cap(int nrhs) {
    if (nrhs <= cap) return;
    ++graph_gen;
    dfree(mmwork);
    mmwork = nullptr;
    if (L() > 1) mmwork = dalloc<zd>(dense_mm_workspace((int)lv.back().n, nrhs));
    dfree(xil); dfree(bil); dfree(xil32); dfree(bil32); dfree(xsw); dfree(xsw32);
    xil = bil = nullptr;
    xil32 = bil32 = nullptr;
    xsw = dalloc<zd>(lv[0].n * nrhs);
    xsw32 = mixed() ? dalloc<zf>(lv[0].n * nrhs) : nullptr;
    if (nrhs >= IL_MIN) {
      xil = dalloc<zd>(lv[0].n * nrhs);
      bil = dalloc<zd>(lv[0].n * nrhs);
      if (mixed()) {
        xil32 = dalloc<zf>(lv[0].n * nrhs);
        bil32 = dalloc<zf>(lv[0].n * nrhs);
      }
    }
    dfree(kpart);
    kpart = nullptr;
    size_t kpart_n = 0;
    for (int l = 0; l < L(); ++l) {
      Level& Lv = lv[l];
      dfree(Lv.x); dfree(Lv.b); dfree(Lv.r);
      dfree(Lv.x32); dfree(Lv.b32); dfree(Lv.r32);
      dfree(Lv.kw); dfree(Lv.kw32); dfree(Lv.kcoef); dfree(Lv.xs); dfree(Lv.xs32);
      Lv.xs = nullptr;
      Lv.xs32 = nullptr;
      Lv.x32 = Lv.b32 = Lv.r32 = nullptr;
      Lv.kw = nullptr;
      Lv.kw32 = nullptr;
      Lv.kcoef = nullptr;
      Lv.x = dalloc<zd>(Lv.n * nrhs);
      Lv.b = dalloc<zd>(Lv.n * nrhs);
      Lv.r = dalloc<zd>(Lv.n * nrhs);
      if (mixed()) {
        Lv.x32 = dalloc<zf>(Lv.n * nrhs);
        Lv.b32 = dalloc<zf>(Lv.n * nrhs);
        Lv.r32 = dalloc<zf>(Lv.n * nrhs);
      }
      if (l >= 1 && !coarsest(l)) {
        Lv.xs = dalloc<zd>(Lv.n * nrhs);
        if (mixed()) Lv.xs32 = dalloc<zf>(Lv.n * nrhs);
      }
      if (kvisited(l)) {
        Lv.kw = dalloc<zd>(5 * Lv.n * nrhs);
        if (mixed()) Lv.kw32 = dalloc<zf>(5 * Lv.n * nrhs);
        Lv.kcoef = dalloc<zd>(4 * (size_t)nrhs);
        kpart_n = std::max(kpart_n, (size_t)kcycle_nblocks(Lv.n) * 2 * nrhs);
      }
    }
    if (kpart_n) kpart = dalloc<zd>(kpart_n);
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
    if (l == 0 && fine_sweeps(f, x, xsw, b, nrhs, 1)) return;
    if (l >= 1 && coarse_pairs(Lv.coarse(), Lv, x, Lv.xs, b, nrhs)) return;
    sweep_colours(l, x, b, nrhs);
  }
  // the sweep as one launch per colour (the reference form of the sweep)
  void sweep_colours(int l, zd* x, const zd* b, int nrhs) {
    Level& Lv = lv[l];
    for (int c = 0; c < Lv.ncol; ++c) {
      if (l == 0) launch_kaczmarz_fine(f, c, Lv.per_colour, x, b, nrhs, s);
      else launch_kaczmarz_coarse(Lv.coarse(), c, Lv.cmode, Lv.per_colour, x, b, nrhs, s);
    }
    check_launch();
  }
  // a coarse sweep as fused colour pairs, alternating between x and xs (an
  // even number of launches, so the last writes x); false if they do not apply
  // (P, xc given: the first launch adds the prolongation P xc to x first)
  bool pairs_ok(const Level& Lv, const void* xs, int nrhs) const {
    return xs && nrhs <= cap && Lv.ncol == 8 && coarse_pair_applies(Lv.ex, Lv.ey, Lv.cmode);
  }
  template <typename T, typename S>
  bool coarse_pairs(const CoarseT<T, S>& c, const Level& Lv, cx<T>* x, cx<T>* xs, const cx<T>* b, int nrhs,
                    const cx<T>* P = nullptr, const cx<T>* xc = nullptr) {
    if (!pairs_ok(Lv, xs, nrhs)) return false;
    cx<T>* a = x;
    cx<T>* o = xs;
    for (int col = 0; col < Lv.ncol; col += 2) {
      launch_kaczmarz_coarse_pair(c, col, Lv.per_colour, a, o, b, nrhs, s, col == 0 ? P : nullptr,
                                  col == 0 ? xc : nullptr);
      std::swap(a, o);
    }
    check_launch();
    return true;
  }
  // count level-0 sweeps blocked in LDS, alternating between x and xs so that
  // the last one writes x (an odd count starts from a copy of x in xs); false
  // if they do not apply.  fz: work carried by the sweeps (FineFuse), the
  // prolongation and the inputs (zero x, FP64 b) by the first, the FP64
  // output by the last (which then writes fz.x64 instead of x); only where
  // fine_fuse_ok
  template <typename T>
  bool fine_sweeps(const FineT<T>& ff, cx<T>* x, cx<T>* xs, const cx<T>* b, int nrhs, int count,
                   const FineFuse<T>& fz = FineFuse<T>{}) {
    if (!xs || nrhs > cap || count < 1 || !fine_sweep_applies(ff, nrhs)) return false;
    if (fz.any() && !fine_sweep_fusable(ff, nrhs)) return false;
    const bool xzero = fz.xzero || fz.b64;
    cx<T>* a = x;
    cx<T>* o = xs;
    if (count & 1) {
      if (!xzero)
        launch_copy(reinterpret_cast<const zd*>(x), reinterpret_cast<zd*>(xs),
                    lv[0].n * nrhs * sizeof(cx<T>) / sizeof(zd), s);
      std::swap(a, o);
    }
    for (int i = 0; i < count; ++i) {
      FineFuse<T> g;
      if (i == 0) {
        g.P = fz.P;
        g.xc = fz.xc;
        g.xzero = fz.xzero;
        g.b64 = fz.b64;
        g.b_out = fz.b_out;
      }
      if (i == count - 1) g.x64 = fz.x64;
      if (!launch_fine_sweep(ff, a, o, b, nrhs, s, g)) throw HipFail("fine sweep: no blocked form for fused work");
      std::swap(a, o);
    }
    check_launch();
    return true;
  }
  // the level-0 sweeps at nrhs run on the interleaved copies: from IL_MIN
  // right-hand sides, but below IL_BLOCKED not where the sweep streamed
  // through LDS (form 2) applies (256^2 x 16 FP32 batches: 9.84 against
  // 10.41 ms; from 32 the interleaved passes win); both give the same bits
  template <typename T>
  bool use_il(const FineT<T>& ff, const cx<T>* xs, const cx<T>* xi, int nrhs) const {
    if (nrhs < IL_MIN || !xi || nrhs > cap) return false;
    if (nrhs >= IL_BLOCKED || !xs || !fine_sweep_applies(ff, nrhs)) return true;
    FineSweepPlan pl;
    int sched[3];
    return fine_sweep_plan_query(ff.N, nrhs, sizeof(T) == 4, 0, pl, sched) != 2;
  }
  // the level-0 sweeps of smooth / smooth32 at nrhs take the LDS-resident
  // blocked form, which carries FineFuse work
  template <typename T>
  bool fine_fuse_ok(const FineT<T>& ff, const cx<T>* xs, const cx<T>* xi, int nrhs) const {
    if (use_il(ff, xs, xi, nrhs)) return false;
    return xs && nrhs <= cap && fine_sweep_applies(ff, nrhs) && fine_sweep_fusable(ff, nrhs);
  }
  // count sweeps on level l; on level 0 through the interleaved copies where
  // use_il, otherwise blocked in LDS where a tile plan applies (the same bits
  // as count calls of sweep)
  // (fz: work the level-0 sweeps carry, only where fine_fuse_ok and count >= 1)
  void smooth(int l, zd* x, const zd* b, int nrhs, int count, const FineFuse<double>& fz = FineFuse<double>{}) {
    if (!fz.any() && l == 0 && use_il(f, xsw, xil, nrhs)) {
      launch_smooth_fine_il(f, lv[0].ncol, lv[0].per_colour, x, b, xil, bil, nrhs, count, s);
      check_launch();
      return;
    }
    if (l == 0 && fine_sweeps(f, x, xsw, b, nrhs, count, fz)) return;
    if (fz.any()) throw HipFail("fine sweeps: fused work where the blocked form does not apply");
    for (int i = 0; i < count; ++i) sweep(l, x, b, nrhs);
  }
  // rc = P^H r; xz (level l+1, may be NULL) = 0 in the same launch
  void restrict_(int l, const zd* r, zd* rc, int nrhs, zd* xz = nullptr) {
    if (l == 0) launch_restrict_fine(f, lv[0].P, r, rc, nrhs, s, xz);
    else launch_restrict_coarse(lv[l].ex, lv[l].ey, lv[l].P, r, rc, nrhs, s, xz);
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
    if (force_mr || !launch_dense_mv_g5(Lv.Ap, Lv.Ablk, (int)Lv.n, b, x, nrhs, Lv.Apart, s))
      launch_dense_mv(Lv.Ainv, (int)Lv.n, b, x, nrhs, force_mr, mmwork, s);
    check_launch();
  }

  // multigrid cycle on level l for A_l x = b, x holds the initial guess
  // (pre-smoothing, residual, restriction, coarse correction, prolongation,
  // post-smoothing; Sec. 1 two-grid scheme applied recursively, Sec. 4)
  // xzero (level 0, where fine_zero_ok): x is zero on entry and is not read
  void cycle(int l, const zd* b, zd* x, int nrhs, bool xzero = false) {
    FineFuse<double> fz0;
    fz0.xzero = xzero;
    if (L() == 1) {  // one level: the cycle reduces to its smoothing sweeps
      smooth(0, x, b, nrhs, p.pre + p.post, fz0);
      return;
    }
    if (coarsest(l)) {
      coarsest_solve(b, x, nrhs);
      return;
    }
    Level& Lv = lv[l];
    Level& C = lv[l + 1];
    smooth(l, x, b, nrhs, p.pre, fz0);
    zd* xz = coarsest(l + 1) ? nullptr : C.x;  // the coarse initial guess x = 0
    // r = b - A x and its restriction, in one launch on level 0 where the
    // lattice takes its tiles and on coarse levels for one right-hand side
    const bool fused = l == 0 ? launch_residual_restrict_fine(f, (const zd*)Lv.P, (const zd*)x, b, C.b, nrhs, s, xz)
                              : nrhs == 1 && launch_residual_restrict_coarse(Lv.coarse(), (const zd*)Lv.P,
                                                                             (const zd*)x, b, C.b, nrhs, s, xz);
    if (!fused) {
      apply(l, x, Lv.r, b, nrhs);
      restrict_(l, Lv.r, C.b, nrhs, xz);
    }
    if (kvisited(l + 1)) {
      kvisit(l + 1, C.b, C.x, nrhs);
    } else {
      const int gamma = (p.cycle == BAMG_CYCLE_W) ? 2 : 1;
      for (int g = 0; g < gamma; ++g) {
        cycle(l + 1, C.b, C.x, nrhs);
        if (coarsest(l + 1)) break;
      }
    }
    if (l >= 1 && p.post >= 1 && pairs_ok(Lv, Lv.xs, nrhs)) {
      // the prolongation inside the first post-smoothing launch
      coarse_pairs(Lv.coarse(), Lv, x, Lv.xs, b, nrhs, (const zd*)Lv.P, (const zd*)C.x);
      smooth(l, x, b, nrhs, p.post - 1);
      return;
    }
    if (l == 0 && p.post >= 1 && fine_fuse_ok(f, xsw, xil, nrhs)) {
      // the prolongation inside the first post-smoothing sweep
      FineFuse<double> fz;
      fz.P = Lv.P;
      fz.xc = C.x;
      smooth(0, x, b, nrhs, p.post, fz);
      return;
    }
    prolong(l, C.x, x, nrhs);
    smooth(l, x, b, nrhs, p.post);
  }
  // the FP64 cycle can start from a zero x it does not read
  bool fine_zero_ok(int nrhs) const {
    return fine_fuse_ok(f, xsw, xil, nrhs) && (L() == 1 ? p.pre + p.post : p.pre) >= 1;
  }

  // K-cycle coarse visit of level c: two steps of flexible GCR on A_c x = r0
  // from x = 0, each preconditioned by one cycle from level c (the sequence of
  // kcycle.hip); x is written whole
  void kvisit(int c, const zd* r0, zd* x, int nrhs) {
    Level& Lv = lv[c];
    const size_t n = Lv.n, nn = n * nrhs;
    zd *z1 = Lv.kw, *w1 = z1 + nn, *r1 = w1 + nn, *z2 = r1 + nn, *w2 = z2 + nn;
    launch_fill_zero(z1, nn, s);
    cycle(c, r0, z1, nrhs);
    apply(c, z1, w1, nullptr, nrhs);
    launch_kdots(w1, w1, r0, n, nrhs, kpart, s);
    launch_kcoef(kpart, n, nrhs, 0, Lv.kcoef, s);
    launch_kstep1(z1, w1, r0, Lv.kcoef, x, r1, n, nrhs, s);
    launch_fill_zero(z2, nn, s);
    cycle(c, r1, z2, nrhs);
    apply(c, z2, w2, nullptr, nrhs);
    launch_kdots(w1, w2, (const zd*)nullptr, n, nrhs, kpart, s);
    launch_kcoef(kpart, n, nrhs, 1, Lv.kcoef, s);
    launch_korth_dots(w2, (const zd*)w1, z2, (const zd*)z1, (const zd*)r1, Lv.kcoef, n, nrhs, kpart, s);
    launch_kcoef(kpart, n, nrhs, 2, Lv.kcoef, s);
    launch_kstep3((const zd*)z2, Lv.kcoef, x, n, nrhs, s);
    check_launch();
  }

  // ------------------------------------------------ mixed-precision cycle
  // The preconditioner of the mixed modes: the same cycle in FP32 with the
  // coarse operators read from their reduced-precision copies and the
  // coarsest level solved with the FP64 inverse (FP64 in and out) or, with
  // coarsest_fp32, with its FP32 copy (FP32 in and out).
  template <typename S>
  CoarseT<float, S> coarse32(int l) const {
    CoarseT<float, S> c;
    c.ex = lv[l].ex; c.ey = lv[l].ey; c.D = (const S*)lv[l].Dst; c.Kinv = lv[l].Kinv32;
    return c;
  }
  template <typename S>
  void apply32(int l, const zf* x, zf* y, const zf* b, int nrhs) {
    if (l == 0) launch_dhat(f32, x, y, b, nrhs, s);
    else if (force_mr || nrhs >= MR_MIN) launch_coarse_apply_mfma(coarse32<S>(l), x, y, b, nrhs, s);
    else launch_coarse_apply(coarse32<S>(l), x, y, b, nrhs, s);
  }
  template <typename S>
  void sweep32(int l, zf* x, const zf* b, int nrhs) {
    Level& Lv = lv[l];
    if (l == 0 && fine_sweeps(f32, x, xsw32, b, nrhs, 1)) return;
    const bool mr = force_mr || nrhs >= MR_MIN;
    if (l >= 1 && !mr && coarse_pairs(coarse32<S>(l), Lv, x, Lv.xs32, b, nrhs)) return;
    sweep_colours32<S>(l, x, b, nrhs, mr);
  }
  // one launch per colour (colour passes on the VALU unless mr)
  template <typename S>
  void sweep_colours32(int l, zf* x, const zf* b, int nrhs, bool mr) {
    Level& Lv = lv[l];
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
  void smooth32(int l, zf* x, const zf* b, int nrhs, int count, const FineFuse<float>& fz = FineFuse<float>{}) {
    if (!fz.any() && l == 0 && use_il(f32, xsw32, xil32, nrhs)) {
      launch_smooth_fine_il(f32, lv[0].ncol, lv[0].per_colour, x, b, xil32, bil32, nrhs, count, s);
      return;
    }
    if (l == 0 && fine_sweeps(f32, x, xsw32, b, nrhs, count, fz)) return;
    if (fz.any()) throw HipFail("fine sweeps: fused work where the blocked form does not apply");
    for (int i = 0; i < count; ++i) sweep32<S>(l, x, b, nrhs);
  }
  // in64, out64 (level 0, where fine_io_ok): x is zero on entry, b is in64
  // rounded to FP32 (the first sweep writes it to b), and the last sweep
  // writes the result to out64 in FP64 instead of to x
  template <typename S>
  void cycle32(int l, const zf* b, zf* x, int nrhs, const zd* in64 = nullptr, zd* out64 = nullptr) {
    FineFuse<float> fin;
    fin.b64 = in64;
    fin.b_out = in64 ? lv[0].b32 : nullptr;
    if (L() == 1) {
      fin.x64 = out64;
      smooth32<S>(0, x, b, nrhs, p.pre + p.post, fin);
      check_launch();
      return;
    }
    if (coarsest(l)) {
      Level& C = lv[l];
      if (nrhs > cap) throw HipFail("coarsest solve: more right-hand sides than the workspace holds");
      if (c32()) {
        if (force_mr || !launch_dense_mv_g5_c32(C.Ap32, C.Ablk, (int)C.n, b, x, nrhs, C.Apart, s))
          launch_dense_mv32(C.Ainv32, (int)C.n, b, x, nrhs, force_mr, (zf*)mmwork, s);
      } else if ((force_mr || !launch_dense_mv_g5_f32io(C.Ap, C.Ablk, (int)C.n, b, x, nrhs, C.Apart, s)) &&
                 !launch_dense_mv_f32io(C.Ainv, (int)C.n, b, x, nrhs, force_mr, s)) {
        launch_convert(b, C.b, C.n * nrhs, s);
        launch_dense_mv(C.Ainv, (int)C.n, C.b, C.x, nrhs, force_mr, mmwork, s);
        launch_convert(C.x, x, C.n * nrhs, s);
      }
      check_launch();
      return;
    }
    Level& Lv = lv[l];
    Level& C = lv[l + 1];
    smooth32<S>(l, x, b, nrhs, p.pre, fin);
    // the restriction also zeroes the coarse initial guess, which the coarsest
    // solve does not need (it writes all of x); the residual and its
    // restriction run in one launch on level 0 where the lattice takes its
    // tiles, and on coarse levels for one right-hand side (the vector form)
    zf* xz = coarsest(l + 1) ? nullptr : C.x32;
    const bool fused =
        l == 0 ? launch_residual_restrict_fine(f32, (const zf*)Lv.P32, (const zf*)x, b, C.b32, nrhs, s, xz)
               : nrhs == 1 && !force_mr &&
                     launch_residual_restrict_coarse(coarse32<S>(l), (const zf*)Lv.P32, (const zf*)x, b, C.b32, nrhs,
                                                     s, xz);
    if (!fused) {
      apply32<S>(l, x, Lv.r32, b, nrhs);
      if (l == 0) launch_restrict_fine(f32, Lv.P32, Lv.r32, C.b32, nrhs, s, xz);
      else launch_restrict_coarse(Lv.ex, Lv.ey, Lv.P32, Lv.r32, C.b32, nrhs, s, xz);
    }
    if (kvisited(l + 1)) {
      kvisit32<S>(l + 1, C.b32, C.x32, nrhs);
    } else {
      const int gamma = (p.cycle == BAMG_CYCLE_W) ? 2 : 1;
      for (int g = 0; g < gamma; ++g) {
        cycle32<S>(l + 1, C.b32, C.x32, nrhs);
        if (coarsest(l + 1)) break;
      }
    }
    if (l >= 1 && p.post >= 1 && !(force_mr || nrhs >= MR_MIN) && pairs_ok(Lv, Lv.xs32, nrhs)) {
      // the prolongation inside the first post-smoothing launch
      coarse_pairs(coarse32<S>(l), Lv, x, Lv.xs32, b, nrhs, (const zf*)Lv.P32, (const zf*)C.x32);
      smooth32<S>(l, x, b, nrhs, p.post - 1);
      check_launch();
      return;
    }
    if (l == 0 && p.post >= 1 && fine_fuse_ok(f32, xsw32, xil32, nrhs)) {
      // the prolongation inside the first post-smoothing sweep, the FP64
      // output (if asked) from the last
      FineFuse<float> fz;
      fz.P = Lv.P32;
      fz.xc = C.x32;
      fz.x64 = out64;
      smooth32<S>(0, x, b, nrhs, p.post, fz);
      check_launch();
      return;
    }
    if (out64) throw HipFail("mixed cycle: FP64 output where the blocked sweep does not apply");
    if (l == 0) launch_prolong_fine(f32, Lv.P32, C.x32, x, nrhs, s);
    else launch_prolong_coarse(Lv.ex, Lv.ey, Lv.P32, C.x32, x, nrhs, s);
    smooth32<S>(l, x, b, nrhs, p.post);
    check_launch();
  }
  // the mixed cycle can take its input and give its output in FP64 through
  // the level-0 sweeps
  bool fine_io_ok(int nrhs) const {
    return fine_fuse_ok(f32, xsw32, xil32, nrhs) && (L() == 1 ? p.pre + p.post >= 1 : (p.pre >= 1 && p.post >= 1));
  }
  // the K-cycle visit of kvisit with FP32 vectors (FP64 sums and coefficients)
  template <typename S>
  void kvisit32(int c, const zf* r0, zf* x, int nrhs) {
    Level& Lv = lv[c];
    const size_t n = Lv.n, nn = n * nrhs;
    zf *z1 = Lv.kw32, *w1 = z1 + nn, *r1 = w1 + nn, *z2 = r1 + nn, *w2 = z2 + nn;
    launch_zero(z1, nn * sizeof(zf), s);
    cycle32<S>(c, r0, z1, nrhs);
    apply32<S>(c, z1, w1, nullptr, nrhs);
    launch_kdots(w1, w1, r0, n, nrhs, kpart, s);
    launch_kcoef(kpart, n, nrhs, 0, Lv.kcoef, s);
    launch_kstep1(z1, w1, r0, Lv.kcoef, x, r1, n, nrhs, s);
    launch_zero(z2, nn * sizeof(zf), s);
    cycle32<S>(c, r1, z2, nrhs);
    apply32<S>(c, z2, w2, nullptr, nrhs);
    launch_kdots(w1, w2, (const zf*)nullptr, n, nrhs, kpart, s);
    launch_kcoef(kpart, n, nrhs, 1, Lv.kcoef, s);
    launch_korth_dots(w2, (const zf*)w1, z2, (const zf*)z1, (const zf*)r1, Lv.kcoef, n, nrhs, kpart, s);
    launch_kcoef(kpart, n, nrhs, 2, Lv.kcoef, s);
    launch_kstep3((const zf*)z2, Lv.kcoef, x, n, nrhs, s);
    check_launch();
  }
  // z = M v for nrhs FP64 level-0 vectors through the FP32 cycle
  // (where the level-0 sweeps are blocked in LDS, the conversions ride in
  // the first and last sweeps)
  void precondition_mixed(const zd* v, zd* z, int nrhs) {
    Level& L0 = lv[0];
    const bool io = fine_io_ok(nrhs);
    if (!io) launch_convert_zero(v, L0.b32, L0.x32, L0.n * nrhs, s);
    const zd* in64 = io ? v : nullptr;
    zd* out64 = io ? z : nullptr;
    switch (p.precision) {
      case BAMG_MIXED_FP16: cycle32<hcx>(0, L0.b32, L0.x32, nrhs, in64, out64); break;
      case BAMG_MIXED_BF16: cycle32<bcx>(0, L0.b32, L0.x32, nrhs, in64, out64); break;
      default: cycle32<zf>(0, L0.b32, L0.x32, nrhs, in64, out64); break;
    }
    if (!io) launch_convert(L0.x32, z, L0.n * nrhs, s);
    check_launch();
  }
  // z = M v in the hierarchy's precision
  void precondition(const zd* v, zd* z, int nrhs) {
    if (mixed()) {
      precondition_mixed(v, z, nrhs);
    } else {
      const bool zero = fine_zero_ok(nrhs);
      if (!zero) launch_fill_zero(z, lv[0].n * nrhs, s);
      cycle(0, v, z, nrhs, zero);
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
    if (!Gst32) Gst32 = dalloc<zf>(nl / 2 * 2);
    launch_slot_gram(f32, Bst32, Gst32, s);
    f32.Gst = Gst32;
    for (int l = 0; l < L(); ++l) {
      Level& Lv = lv[l];
      if (Lv.P) {
        if (!Lv.P32) Lv.P32 = dalloc<zf>(Lv.n * 8);
        launch_convert(Lv.P, Lv.P32, Lv.n * 8, s);
      }
      if (coarsest(l) && L() > 1 && c32()) {
        if (Lv.n % 16 != 0 || dense_mm32_workspace_bytes((int)Lv.n, cap) > dense_mm_workspace((int)Lv.n, cap) * sizeof(zd))
          throw HipFail("coarsest level: FP32 inverse needs n % 16 == 0 and the split-K workspace");
        if (!Lv.Ainv32) Lv.Ainv32 = dalloc<zf>(Lv.n * Lv.n);
        launch_convert(Lv.Ainv, Lv.Ainv32, Lv.n * Lv.n, s);
        if (Lv.Ap) {
          const size_t nbk = Lv.n / 64;
          if (!Lv.Ap32) Lv.Ap32 = dalloc<zf>(nbk * (nbk + 1) / 2 * 64 * 64);
          launch_pack_g5_f32(Lv.Ainv, (int)Lv.n, Lv.Ablk, Lv.Ap32, s);
        }
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
    if (C.Ap) launch_pack_g5(C.Ainv, n, C.Ablk, C.Ap, s);
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

  // ---------------------------------------------------------- bootstrap cycles
  // The bootstrap setup of Sec. 3.4 with the multigrid eigensolver, in the
  // Hermitian form of Theorem 1 (Z_l = Gamma_5 D_l, T_l = I): relaxation test
  // vectors V^r on Z v = 0, eigenvector approximations V^e on Z v = lambda v
  // (Kaczmarz on (D_l - lambda Gamma_5) v = 0, Ritz value after every sweep),
  // the k_e eigenpairs of Z_L with the smallest |lambda| on the coarsest
  // level, least squares P from V^r and V^e together.  Node kinds and their
  // order follow the setup-cycle figure of Sec. 3.5 (see boot_visit).
  zd* tve(int l) { return lv[l].tv + lv[l].n * p.n_tv; }

  void normalise(int l, zd* X, int k) {
    const size_t n = lv[l].n;
    launch_norms(X, n, k, n, partial, hdev, s);
    launch_normalize(X, n, k, n, hdev, s);
    check_launch();
  }
  // one Kaczmarz sweep on (A_l - lam_r Gamma_5) x_r = 0 for k vectors
  void sweep_shift(int l, zd* X, const double* lam, int k) {
    Level& Lv = lv[l];
    for (int c = 0; c < Lv.ncol; ++c) {
      if (l == 0) launch_kaczmarz_fine(f, c, Lv.per_colour, X, (const zd*)nullptr, k, s, lam);
      else launch_kaczmarz_coarse_shift(Lv.coarse(), c, Lv.cmode, Lv.per_colour, X, lam, k, s);
    }
    check_launch();
  }
  // lam[r] = <Z_l x_r, x_r> / <x_r, x_r> (eq. eqevZ, T = I)
  void ritz(int l, const zd* X, int k, double* lam) {
    Level& Lv = lv[l];
    apply(l, X, Lv.r, nullptr, k);
    launch_ritz(X, Lv.r, Lv.n, Lv.dps, k, partial, lam, s);
    check_launch();
  }
  void boot_relax_r(int l, int nu) {
    for (int i = 0; i < nu; ++i) sweep(l, lv[l].tv, nullptr, p.n_tv);
    normalise(l, lv[l].tv, p.n_tv);
  }
  void boot_relax_e(int l, int nu) {
    if (!have_e) return;
    for (int i = 0; i < nu; ++i) {
      sweep_shift(l, tve(l), lam_dev, ke);
      ritz(l, tve(l), ke, lam_dev);
    }
    normalise(l, tve(l), ke);
  }
  void boot_fit(int l) {
    Level& Lv = lv[l];
    const int k = p.n_tv + (have_e ? ke : 0);
    if (k <= 8) fit(l, Lv.tv);
    else launch_fit_ls(l == 0, Lv.ex, Lv.ey, Lv.tv, k, Lv.P, s);
    check_launch();
    build_next(l);
    restrict_(l, Lv.tv, lv[l + 1].tv, k);
  }
  void boot_interp_e(int l) {
    launch_fill_zero(tve(l), lv[l].n * ke, s);
    prolong(l, tve(l + 1), tve(l), ke);
  }
  // Hermitian eigen-decomposition of a small host matrix by cyclic Jacobi
  // rotations (w unsorted, E columns = eigenvectors)
  static void small_heig(int n, std::vector<std::complex<double>>& H, std::vector<double>& w,
                         std::vector<std::complex<double>>& E) {
    typedef std::complex<double> Cd;
    E.assign((size_t)n * n, Cd(0.0));
    for (int i = 0; i < n; ++i) E[(size_t)i * n + i] = 1.0;
    double fro = 0;
    for (auto& z : H) fro += std::norm(z);
    for (int sweep = 0; sweep < 100; ++sweep) {
      double off = 0;
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
          if (i != j) off += std::norm(H[(size_t)i * n + j]);
      if (off <= 1e-30 * fro || off == 0.0) break;
      for (int a = 0; a < n - 1; ++a)
        for (int b = a + 1; b < n; ++b) {
          const Cd hab = H[(size_t)a * n + b];
          const double r = std::abs(hab);
          if (r == 0.0) continue;
          const Cd ph = hab / r;
          const double ta = (H[(size_t)b * n + b].real() - H[(size_t)a * n + a].real()) / (2.0 * r);
          const double t = (ta >= 0 ? 1.0 : -1.0) / (std::abs(ta) + std::sqrt(1.0 + ta * ta));
          const double c = 1.0 / std::sqrt(1.0 + t * t), sn = t * c;
          const Cd u00 = c, u01 = sn, u10 = -sn * std::conj(ph), u11 = c * std::conj(ph);
          for (int k = 0; k < n; ++k) {
            const Cd x0 = H[(size_t)k * n + a], x1 = H[(size_t)k * n + b];
            H[(size_t)k * n + a] = x0 * u00 + x1 * u10;
            H[(size_t)k * n + b] = x0 * u01 + x1 * u11;
          }
          for (int k = 0; k < n; ++k) {
            const Cd x0 = H[(size_t)a * n + k], x1 = H[(size_t)b * n + k];
            H[(size_t)a * n + k] = std::conj(u00) * x0 + std::conj(u10) * x1;
            H[(size_t)b * n + k] = std::conj(u01) * x0 + std::conj(u11) * x1;
          }
          H[(size_t)a * n + b] = 0.0;
          H[(size_t)b * n + a] = 0.0;
          for (int k = 0; k < n; ++k) {
            const Cd x0 = E[(size_t)k * n + a], x1 = E[(size_t)k * n + b];
            E[(size_t)k * n + a] = x0 * u00 + x1 * u10;
            E[(size_t)k * n + b] = x0 * u01 + x1 * u11;
          }
        }
    }
    w.resize(n);
    for (int i = 0; i < n; ++i) w[i] = H[(size_t)i * n + i].real();
  }
  // G = X^H Y for pc vectors of length n (device), result on the host (column j: X^H Y_j)
  void block_gram(const zd* X, const zd* Y, size_t n, int pc, std::vector<std::complex<double>>& G) {
    for (int j = 0; j < pc; ++j) launch_multidot(X, n, pc, Y + (size_t)j * n, n, partial, eigC + (size_t)j * pc, s);
    check_launch();
    HIPCHK(hipMemcpyAsync(eigH, eigC, (size_t)pc * pc * sizeof(zd), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    G.assign((size_t)pc * pc, 0.0);
    for (int j = 0; j < pc; ++j)
      for (int i = 0; i < pc; ++i) G[(size_t)i * pc + j] = {eigH[(size_t)j * pc + i].x, eigH[(size_t)j * pc + i].y};
  }
  // Y = X C with the host pc x pc matrix C
  void block_combine(const zd* X, const std::vector<std::complex<double>>& Cm, zd* Y, size_t n, int pc) {
    for (size_t e = 0; e < (size_t)pc * pc; ++e) eigH[e] = zd{Cm[e].real(), Cm[e].imag()};
    HIPCHK(hipMemcpyAsync(eigW, eigH, (size_t)pc * pc * sizeof(zd), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));  // eigH is reused by the next host step
    launch_block_combine(X, eigW, Y, n, pc, s);
    check_launch();
  }
  // eigX <- an orthonormal basis of the pc vectors `in` (Cholesky QR applied
  // twice; `in` and `work` are overwritten, neither may be eigX unless in == eigX)
  void cholqr2(zd* in, zd* work, size_t n, int pc) {
    typedef std::complex<double> Cd;
    for (int pass = 0; pass < 2; ++pass) {
      const zd* src = pass == 0 ? in : work;
      zd* dst = pass == 0 ? work : eigX;
      std::vector<Cd> G;
      block_gram(src, src, n, pc, G);
      // G = L L^H, then dst = src L^{-H}
      std::vector<Cd> Lm((size_t)pc * pc, 0.0);
      for (int j = 0; j < pc; ++j) {
        double d = G[(size_t)j * pc + j].real();
        for (int k = 0; k < j; ++k) d -= std::norm(Lm[(size_t)j * pc + k]);
        if (!(d > 0)) throw BadArg("coarsest eigensolver: rank-deficient block");
        const double ljj = std::sqrt(d);
        Lm[(size_t)j * pc + j] = ljj;
        for (int i = j + 1; i < pc; ++i) {
          Cd sum = G[(size_t)i * pc + j];
          for (int k = 0; k < j; ++k) sum -= Lm[(size_t)i * pc + k] * std::conj(Lm[(size_t)j * pc + k]);
          Lm[(size_t)i * pc + j] = sum / ljj;
        }
      }
      // Ci = L^{-H} (upper triangular): L^H Ci = I column by column
      std::vector<Cd> Ci((size_t)pc * pc, 0.0);
      for (int c = 0; c < pc; ++c)
        for (int i = pc - 1; i >= 0; --i) {
          Cd sum = (i == c) ? Cd(1.0) : Cd(0.0);
          for (int k = i + 1; k < pc; ++k) sum -= std::conj(Lm[(size_t)k * pc + i]) * Ci[(size_t)k * pc + c];
          Ci[(size_t)i * pc + c] = sum / Lm[(size_t)i * pc + i].real();
        }
      block_combine(src, Ci, dst, n, pc);
    }
  }
  // the ke eigenpairs of Z_L = Gamma_5 D_L with the smallest |lambda| by block
  // inverse iteration with Z_L^{-1} = A_L^{-1} Gamma_5 (the coarsest inverse)
  // and Rayleigh-Ritz on 2 ke vectors, until the residuals |Z x - lambda x| of
  // the ke Ritz pairs are below 1e-12 max |lambda| (or 500 iterations)
  void boot_coarsest(zd* out = nullptr) {
    typedef std::complex<double> Cd;
    Level& C = lv.back();
    const size_t n = C.n;
    const int pc = (int)std::min<size_t>((size_t)2 * ke, n);
    launch_philox_tv((int)n, pc, p.seed ^ 0x3c6ef372fe94f82bull, eigX, s);
    cholqr2(eigX, eigY, n, pc);  // eigX <- orthonormal
    std::vector<double> vals, sorted(pc);
    std::vector<Cd> H, E, G;
    for (int it = 0; it < 500; ++it) {
      launch_gamma5(eigX, eigT, n, 16, pc, s);
      launch_dense_mv(C.Ainv, (int)n, eigT, eigY, pc, true, eigmm, s);
      check_launch();
      cholqr2(eigY, eigT, n, pc);  // eigX <- orthonormal basis of A^{-1} Gamma_5 X
      launch_coarse_apply(C.coarse(), (const zd*)eigX, eigT, (const zd*)nullptr, pc, s);
      launch_gamma5(eigT, eigY, n, 16, pc, s);  // eigY = Z X
      check_launch();
      block_gram(eigX, eigY, n, pc, H);  // X^H Z X
      for (int i = 0; i < pc; ++i)       // symmetrise the rounding
        for (int j = i + 1; j < pc; ++j) {
          const Cd a = 0.5 * (H[(size_t)i * pc + j] + std::conj(H[(size_t)j * pc + i]));
          H[(size_t)i * pc + j] = a;
          H[(size_t)j * pc + i] = std::conj(a);
        }
      for (int i = 0; i < pc; ++i) H[(size_t)i * pc + i] = H[(size_t)i * pc + i].real();
      small_heig(pc, H, vals, E);
      std::vector<int> idx(pc);
      for (int i = 0; i < pc; ++i) idx[i] = i;
      std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return std::abs(vals[a]) < std::abs(vals[b]); });
      std::vector<Cd> W((size_t)pc * pc);
      for (int i = 0; i < pc; ++i)
        for (int j = 0; j < pc; ++j) W[(size_t)i * pc + j] = E[(size_t)i * pc + idx[j]];
      for (int j = 0; j < pc; ++j) sorted[j] = vals[idx[j]];
      // Ritz vectors X W (into eigT), Z X W (into eigX), residuals of the first ke (into eigR)
      block_combine(eigX, W, eigT, n, pc);
      block_combine(eigY, W, eigX, n, pc);
      for (int j = 0; j < ke; ++j) lam_host[j] = sorted[j];
      HIPCHK(hipMemcpyAsync(lam_dev, lam_host, ke * sizeof(double), hipMemcpyHostToDevice, s));
      launch_eig_residual(eigX, eigT, lam_dev, eigR, n, ke, s);
      launch_norms(eigR, n, ke, n, partial, eigC, s);
      check_launch();
      HIPCHK(hipMemcpyAsync(eigH, eigC, ke * sizeof(zd), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      std::swap(eigX, eigT);  // eigX = Ritz vectors
      double res = 0, scale = 0;
      for (int j = 0; j < ke; ++j) {
        res = std::max(res, std::sqrt(eigH[j].x));
        scale = std::max(scale, std::abs(sorted[j]));
      }
      if (res <= 1e-12 * scale) break;
    }
    // V^e on the coarsest level: the ke Ritz vectors of smallest |lambda| (unit norm)
    launch_copy(eigX, out ? out : tve((int)lv.size() - 1), n * ke, s);
    check_launch();
    have_e = true;
  }
  void boot_arrive(int l, int nu, bool first) {
    boot_relax_r(l, nu);
    if (!first) boot_relax_e(l, nu);
    boot_fit(l);
  }
  // a visit of level l >= 1 in a setup cycle: arrive, then gamma visits of the
  // level below, each followed by the interpolation of V^e; between two visits
  // the level relaxes both sets and recomputes P, after the last it relaxes V^e
  void boot_visit(int l, const std::vector<int>& nu, bool first, int gamma) {
    const int Lc = L() - 1;
    boot_arrive(l, nu[l], first);
    for (int g = 0; g < gamma; ++g) {
      if (l + 1 == Lc) boot_coarsest();
      else boot_visit(l + 1, nu, first && g == 0, gamma);
      boot_interp_e(l);
      if (g < gamma - 1) boot_arrive(l, nu[l], false);
      else boot_relax_e(l, nu[l]);
    }
  }
  void boot_cycle(const std::vector<int>& nu, bool first, int gamma) {
    boot_arrive(0, nu[0], first);
    if (L() == 2) boot_coarsest();
    else boot_visit(1, nu, first, gamma);
    boot_interp_e(0);
    boot_relax_e(0, nu[0]);
  }
  zd* eigmm = nullptr;
  // buffers of the eigensolver for ke_ (<= 8) eigenpairs
  void ensure_boot(int ke_) {
    if (lam_dev) return;
    ke = ke_;
    const size_t nL = lv.back().n;
    const int pc = (int)std::min<size_t>((size_t)2 * 8, nL);
    lam_dev = dalloc<double>(16);
    HIPCHK(hipHostMalloc((void**)&lam_host, 16 * sizeof(double)));
    eigX = dalloc<zd>(nL * pc);
    eigY = dalloc<zd>(nL * pc);
    eigT = dalloc<zd>(nL * pc);
    eigR = dalloc<zd>(nL * pc);
    eigC = dalloc<zd>((size_t)pc * pc);
    eigW = dalloc<zd>((size_t)pc * pc);
    eigmm = dalloc<zd>(dense_mm_workspace((int)nL, pc));
    HIPCHK(hipHostMalloc((void**)&eigH, (size_t)pc * pc * sizeof(zd)));
  }
  void boot_setup() {
    ensure_boot(p.n_ev);
    ke = p.n_ev;
    have_e = false;
    const int gamma = (p.setup_mode == 1) ? 2 : 1;
    auto sweeps = [&](int mu) {
      std::vector<int> nu(L());
      for (int l = 0; l < L(); ++l) nu[l] = (p.setup_mode == 1) ? mu : mu * (1 << l);
      return nu;
    };
    boot_cycle(sweeps(p.boot_nu1), true, gamma);
    // adaptive step (Sec. 4.1): two cycles of the current solver on Dhat v = 0
    // for the eigenvector approximation with the smallest |Ritz value|
    HIPCHK(hipMemcpyAsync(lam_host, lam_dev, ke * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    int kmin = 0;
    for (int k = 1; k < ke; ++k)
      if (std::abs(lam_host[k]) < std::abs(lam_host[kmin])) kmin = k;
    Level& L0 = lv[0];
    zd* v = tve(0) + L0.n * kmin;
    launch_fill_zero(L0.b, L0.n, s);
    for (int c = 0; c < 2; ++c) cycle(0, L0.b, v, 1);
    normalise(0, v, 1);
    ritz(0, v, 1, lam_dev + kmin);
    boot_cycle(sweeps(p.boot_nu2), false, gamma);
    launch_copy(L0.tv, tvsave, L0.n * p.n_tv, s);
    HIPCHK(hipMemcpyAsync(lam_host, lam_dev, ke * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    lam_final.assign(lam_host, lam_host + ke);
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
