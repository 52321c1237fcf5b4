// CPU FP64 reference oracle for the odd-even reduced 2D Wilson-Dirac
// bootstrap-AMG solve path (Brannick & Kahl, "Bootstrap Algebraic Multigrid
// for the 2D Wilson Dirac system", arXiv:1308.5992).
//
// TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
// statement of what the GPU library computes.  It shares no code, header,
// table or helper with the HIP path; only the test-suite, the smoke check and
// the CPU-baseline leg of the benchmark may load it.  Everything is FP64,
// std::complex<double>, single-threaded loops over explicit sparse (CSR) or
// dense matrices built from the paper's definitions.
//
// Readings of the paper that the code below takes:
//   * Wilson operator: eq. (wilson) of Sec. 2 with m_q = m + 2 in 2D, the
//     gamma matrices of Sec. 2 and U(1) links; the link sits on the forward
//     hop and its conjugate on the backward hop exactly as eq. (wilson) says.
//   * Odd-even reduction (Sec. 3.2, eq. wilsonSchur): with c = m + 2,
//     Dhat = (D_ee - D_eo D_oo^{-1} D_oe)/c = I - c^{-2} H_eo H_oe,
//     bhat = b_e/c + c^{-2} H_eo b_o, x_o = b_o/c + c^{-1} H_oe x_e.
//   * Kaczmarz (Sec. 3.1): row projection x += (r_i/||d_i||^2) d_i^H with
//     relaxation weight one, rows ordered by a multicolouring (Sec. 3.1 says a
//     colouring exists but does not give one): 16 colours on the fine even
//     grid, 8 (or 16) colours on coarse grids.
//   * Least squares interpolation (Sec. 3.3, eq. LSfuncrowi) applied per
//     aggregate and spin: with k <= 8 test vectors on a 16-dof block the fit
//     is exact and P_{a,s} is the orthonormal basis from classical
//     Gram-Schmidt with re-orthogonalisation (R_jj > 0) of the test vectors.
//   * Spin-block P (Sec. 3.5, eq. bs) so that restriction is P^H and the
//     coarse operator is the Galerkin product P^H D P (Sec. 3.5).
//   * Coarsest grid solved directly (Sec. 4): dense LU with partial pivoting.
//   * Outer Krylov (Sec. 4): flexible GMRES(32) right-preconditioned by one
//     multigrid cycle, classical Gram-Schmidt applied twice, Givens rotations.
//   * Cycles: the two-grid scheme of Sec. 1 applied recursively with gamma = 1
//     (V) or gamma = 2 (W, the solve cycle of Sec. 4) coarse visits; the
//     K-cycle option replaces the coarse visit of every level whose coarser
//     neighbour is not the coarsest by two steps of flexible GCR on the coarse
//     system, each preconditioned by one cycle from that level (the paper
//     names no Krylov-accelerated cycle; this is the recursive Krylov cycle of
//     the multigrid literature, with a fixed two steps).
//   * Stand-alone convergence rate (Sec. 4): rho = ||e^nu|| / ||e^{nu-1}|| of
//     the iteration x <- x + M (b - Dhat x) with M one cycle, on b = 0.
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>
#include <memory>

typedef std::complex<double> cplx;

namespace {

// ---------------------------------------------------------------------------
// Sparse matrix (CSR).  Rows and columns index degrees of freedom.
// ---------------------------------------------------------------------------
struct CSR {
  int nr = 0, nc = 0;
  std::vector<int> ptr, col;
  std::vector<cplx> val;
};

// y = A x
void csr_mv(const CSR& A, const cplx* x, cplx* y) {
  for (int r = 0; r < A.nr; ++r) {
    cplx s = 0.0;
    for (int p = A.ptr[r]; p < A.ptr[r + 1]; ++p) s += A.val[p] * x[A.col[p]];
    y[r] = s;
  }
}

// conjugate transpose
CSR csr_adjoint(const CSR& A) {
  CSR T; T.nr = A.nc; T.nc = A.nr;
  T.ptr.assign(T.nr + 1, 0);
  for (int p = 0; p < (int)A.col.size(); ++p) T.ptr[A.col[p] + 1]++;
  for (int r = 0; r < T.nr; ++r) T.ptr[r + 1] += T.ptr[r];
  T.col.resize(A.col.size()); T.val.resize(A.val.size());
  std::vector<int> fill(T.ptr.begin(), T.ptr.end() - 1);
  for (int r = 0; r < A.nr; ++r)
    for (int p = A.ptr[r]; p < A.ptr[r + 1]; ++p) {
      int q = fill[A.col[p]]++;
      T.col[q] = r; T.val[q] = std::conj(A.val[p]);
    }
  return T;
}

// C = A B (row-wise with a dense accumulator).  Structural entries are kept
// even when their value cancels to zero, so the pattern is the product pattern.
CSR csr_mul(const CSR& A, const CSR& B) {
  CSR C; C.nr = A.nr; C.nc = B.nc; C.ptr.assign(C.nr + 1, 0);
  std::vector<int> mark(B.nc, -1);
  std::vector<cplx> acc(B.nc, 0.0);
  std::vector<int> cols;
  for (int r = 0; r < A.nr; ++r) {
    cols.clear();
    for (int p = A.ptr[r]; p < A.ptr[r + 1]; ++p) {
      int k = A.col[p];
      for (int q = B.ptr[k]; q < B.ptr[k + 1]; ++q) {
        int c = B.col[q];
        if (mark[c] != r) { mark[c] = r; acc[c] = 0.0; cols.push_back(c); }
        acc[c] += A.val[p] * B.val[q];
      }
    }
    std::sort(cols.begin(), cols.end());
    for (int c : cols) { C.col.push_back(c); C.val.push_back(acc[c]); }
    C.ptr[r + 1] = (int)C.col.size();
  }
  return C;
}

// ---------------------------------------------------------------------------
// Lattice, gauge field and the Wilson operator (Sec. 2, eq. wilson).
// Full-lattice field layout: psi[(y*N + x)*2 + s].  Links: U[(mu*N + y)*N + x],
// mu = 0 the link (x,y)->(x+1,y), mu = 1 the link (x,y)->(x,y+1).
// ---------------------------------------------------------------------------
inline int wrap(int a, int n) { return ((a % n) + n) % n; }
inline int fmod_floor(int a, int n) { return ((a % n) + n) % n; }

struct Mat2 { cplx a[2][2]; };

// P_mu^{+/-} = (I +/- gamma_mu)/2 with gamma_1 = [[0,1],[1,0]],
// gamma_2 = [[0,i],[-i,0]] (Sec. 2).
Mat2 proj(int mu, int sign) {
  const cplx I(0.0, 1.0);
  cplx g[2][2];
  if (mu == 0) { g[0][0] = 0.0; g[0][1] = 1.0; g[1][0] = 1.0; g[1][1] = 0.0; }
  else { g[0][0] = 0.0; g[0][1] = I; g[1][0] = -I; g[1][1] = 0.0; }
  Mat2 P;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      P.a[i][j] = 0.5 * ((i == j ? 1.0 : 0.0) + (double)sign * g[i][j]);
  return P;
}

// Hopping matrix H of the full lattice, D = (m+2) I - H:
// (H psi)_z = sum_mu [ P_mu^- U_mu(z) psi_{z+mu} + P_mu^+ conj(U_mu(z-mu)) psi_{z-mu} ]
CSR build_hop(int N, const cplx* U) {
  CSR H; H.nr = H.nc = 2 * N * N; H.ptr.assign(H.nr + 1, 0);
  Mat2 Pm[2] = {proj(0, -1), proj(1, -1)};
  Mat2 Pp[2] = {proj(0, +1), proj(1, +1)};
  for (int y = 0; y < N; ++y)
    for (int x = 0; x < N; ++x) {
      int z = y * N + x;
      for (int s = 0; s < 2; ++s) {
        // collect (col, val) pairs for row (z, s)
        std::vector<std::pair<int, cplx>> ent;
        for (int mu = 0; mu < 2; ++mu) {
          int xf = mu == 0 ? wrap(x + 1, N) : x, yf = mu == 1 ? wrap(y + 1, N) : y;
          int xb = mu == 0 ? wrap(x - 1, N) : x, yb = mu == 1 ? wrap(y - 1, N) : y;
          cplx uf = U[(mu * N + y) * N + x];
          cplx ub = std::conj(U[(mu * N + yb) * N + xb]);
          for (int t = 0; t < 2; ++t) {
            ent.push_back({(yf * N + xf) * 2 + t, Pm[mu].a[s][t] * uf});
            ent.push_back({(yb * N + xb) * 2 + t, Pp[mu].a[s][t] * ub});
          }
        }
        std::sort(ent.begin(), ent.end(), [](auto& a, auto& b) { return a.first < b.first; });
        // merge duplicates (only possible on tiny lattices)
        for (size_t i = 0; i < ent.size(); ++i) {
          if (!H.col.empty() && (int)H.col.size() > H.ptr[2 * z + s] && H.col.back() == ent[i].first)
            H.val.back() += ent[i].second;
          else { H.col.push_back(ent[i].first); H.val.push_back(ent[i].second); }
        }
        H.ptr[2 * z + s + 1] = (int)H.col.size();
      }
    }
  return H;
}

// Even sites in half-x order: e = y*(N/2) + xh with x = 2*xh + (y mod 2).
// Odd sites in half-x order: o = y*(N/2) + xh with x = 2*xh + 1 - (y mod 2).
int even_site_x(int xh, int y) { return 2 * xh + (y & 1); }
int odd_site_x(int xh, int y) { return 2 * xh + 1 - (y & 1); }

// Selection of the rows/cols of the full hop matrix: returns the block H_{AB}
// with rows on parity A and cols on parity B (0 even, 1 odd), both in half-x order.
CSR hop_block(int N, const CSR& H, int prow, int pcol) {
  int half = N / 2;
  std::vector<int> full2red(N * N, -1);
  for (int y = 0; y < N; ++y)
    for (int xh = 0; xh < half; ++xh) {
      int x = pcol == 0 ? even_site_x(xh, y) : odd_site_x(xh, y);
      full2red[y * N + x] = y * half + xh;
    }
  CSR B; B.nr = B.nc = N * N; B.ptr.assign(B.nr + 1, 0);
  for (int y = 0; y < N; ++y)
    for (int xh = 0; xh < half; ++xh) {
      int x = prow == 0 ? even_site_x(xh, y) : odd_site_x(xh, y);
      int zr = y * half + xh, zf = y * N + x;
      for (int s = 0; s < 2; ++s) {
        int r = 2 * zf + s;
        for (int p = H.ptr[r]; p < H.ptr[r + 1]; ++p) {
          int cs = H.col[p] / 2, ct = H.col[p] % 2;
          int red = full2red[cs];
          if (red < 0) continue;  // entry in the other parity (absent for N even)
          B.col.push_back(2 * red + ct); B.val.push_back(H.val[p]);
        }
        B.ptr[2 * zr + s + 1] = (int)B.col.size();
      }
    }
  return B;
}

struct Problem {
  int N; double m, c;
  std::vector<cplx> U;
  CSR H, Heo, Hoe, Dhat;
};

void build_problem(Problem& P, int N, const double* U, double m) {
  P.N = N; P.m = m; P.c = m + 2.0;
  P.U.assign((const cplx*)U, (const cplx*)U + 2 * N * N);
  P.H = build_hop(N, P.U.data());
  P.Heo = hop_block(N, P.H, 0, 1);
  P.Hoe = hop_block(N, P.H, 1, 0);
  CSR HH = csr_mul(P.Heo, P.Hoe);
  // Dhat = I - c^{-2} H_eo H_oe
  CSR D; D.nr = D.nc = HH.nr; D.ptr.assign(D.nr + 1, 0);
  double k2 = 1.0 / (P.c * P.c);
  for (int r = 0; r < HH.nr; ++r) {
    bool diag = false;
    for (int p = HH.ptr[r]; p < HH.ptr[r + 1]; ++p) {
      cplx v = -k2 * HH.val[p];
      if (HH.col[p] == r) { v += 1.0; diag = true; }
      D.col.push_back(HH.col[p]); D.val.push_back(v);
    }
    if (!diag) {  // keep rows sorted
      auto it = std::lower_bound(D.col.begin() + D.ptr[r], D.col.end(), r);
      size_t off = it - D.col.begin();
      D.col.insert(it, r); D.val.insert(D.val.begin() + off, 1.0);
    }
    D.ptr[r + 1] = (int)D.col.size();
  }
  P.Dhat = D;
}

// ---------------------------------------------------------------------------
// Multicolour orderings (Sec. 3.1).
// Fine even site (x,y): u = (x+y)/2, v = (x-y)/2, colour = 4*(u mod 4) + (v mod 4).
// Coarse site (ax, ay) on an ex x ey grid: if both extents are multiples of 8,
// colour = (ax - 3 ay) mod 8; else if multiples of 4, colour = 4*(ay mod 4) +
// (ax mod 4); else every site is its own colour.
// ---------------------------------------------------------------------------
int fine_colour(int x, int y) {
  int u = (x + y) / 2;
  int v = (x - y);  // even
  v = (v >= 0) ? v / 2 : -((-v) / 2);
  return 4 * fmod_floor(u, 4) + fmod_floor(v, 4);
}

int coarse_ncolours(int ex, int ey) {
  if (ex % 8 == 0 && ey % 8 == 0) return 8;
  if (ex % 4 == 0 && ey % 4 == 0) return 16;
  return ex * ey;
}
int coarse_colour(int ax, int ay, int ex, int ey) {
  if (ex % 8 == 0 && ey % 8 == 0) return fmod_floor(ax - 3 * ay, 8);
  if (ex % 4 == 0 && ey % 4 == 0) return 4 * (ay % 4) + (ax % 4);
  return ay * ex + ax;
}

// ---------------------------------------------------------------------------
// Level of the hierarchy.  Level 1 is Dhat on the half-x even grid (2 dofs per
// site); level l > 1 lives on an ex x ey grid of aggregates with 16 dofs per
// site, dof 8*s + k carrying spin s.
// ---------------------------------------------------------------------------
struct Level {
  int ex, ey, dps;          // grid extents (sites) and dofs per site
  CSR A;                    // operator
  std::vector<double> nu;   // squared row norms ||d_r||^2
  std::vector<int> order;   // Kaczmarz row order
  // interpolation to this level from the next coarser one (absent on the coarsest)
  int cx = 0, cy = 0;       // coarse grid extents
  int ax = 0, ay = 0;       // aggregate shape in sites of this level
  int rows_per = 0;         // rows of P_{a,s}: sites per aggregate * dofs per spin
  std::vector<cplx> Pblk;   // [agg][s][row][k], k < 8
  CSR P, PH;
  // dense LU of the coarsest operator
  std::vector<cplx> LU; std::vector<int> piv; bool singular = false;
};

void level_norms_and_order(Level& L, bool fine, int N) {
  L.nu.assign(L.A.nr, 0.0);
  for (int r = 0; r < L.A.nr; ++r)
    for (int p = L.A.ptr[r]; p < L.A.ptr[r + 1]; ++p) L.nu[r] += std::norm(L.A.val[p]);
  L.order.clear();
  if (fine) {
    int half = N / 2;
    for (int col = 0; col < 16; ++col)
      for (int y = 0; y < N; ++y)
        for (int xh = 0; xh < half; ++xh)
          if (fine_colour(even_site_x(xh, y), y) == col)
            for (int s = 0; s < 2; ++s) L.order.push_back(2 * (y * half + xh) + s);
  } else {
    int nc = coarse_ncolours(L.ex, L.ey);
    for (int col = 0; col < nc; ++col)
      for (int ay = 0; ay < L.ey; ++ay)
        for (int ax = 0; ax < L.ex; ++ax)
          if (coarse_colour(ax, ay, L.ex, L.ey) == col)
            for (int d = 0; d < L.dps; ++d) L.order.push_back((ay * L.ex + ax) * L.dps + d);
  }
}

// One forward Kaczmarz sweep (row projection) on A x = b in the level's order.
void kaczmarz_sweep(const Level& L, cplx* x, const cplx* b) {
  const CSR& A = L.A;
  for (int r : L.order) {
    if (L.nu[r] == 0.0) continue;
    cplx res = b ? b[r] : cplx(0.0);
    for (int p = A.ptr[r]; p < A.ptr[r + 1]; ++p) res -= A.val[p] * x[A.col[p]];
    cplx alpha = res / L.nu[r];
    for (int p = A.ptr[r]; p < A.ptr[r + 1]; ++p) x[A.col[p]] += alpha * std::conj(A.val[p]);
  }
}

// Aggregation maps.  Level 1: 4x4 blocks of the half-x grid, local site order
// (y, then xh).  Level l > 1: 2x2 blocks of sites, local order (ay, then ax).
// fine_dof -> (aggregate, spin, row within P_{a,s})
struct AggMap { std::vector<int> agg, spin, row; };

AggMap aggregate_map(const Level& F, bool fine) {
  AggMap M; int n = F.A.nr;
  M.agg.resize(n); M.spin.resize(n); M.row.resize(n);
  for (int sy = 0; sy < F.ey; ++sy)
    for (int sx = 0; sx < F.ex; ++sx) {
      int site = sy * F.ex + sx;
      int a = (sy / F.ay) * F.cx + (sx / F.ax);
      int loc = (sy % F.ay) * F.ax + (sx % F.ax);
      for (int d = 0; d < F.dps; ++d) {
        int dof = site * F.dps + d;
        M.agg[dof] = a;
        if (fine) { M.spin[dof] = d; M.row[dof] = loc; }
        else { M.spin[dof] = d / 8; M.row[dof] = 8 * loc + (d % 8); }
      }
    }
  return M;
}

void build_P_csr(Level& F, bool fine) {
  AggMap M = aggregate_map(F, fine);
  int n = F.A.nr;
  F.P.nr = n; F.P.nc = F.cx * F.cy * 16; F.P.ptr.assign(n + 1, 0);
  F.P.col.clear(); F.P.val.clear();
  for (int dof = 0; dof < n; ++dof) {
    int a = M.agg[dof], s = M.spin[dof], r = M.row[dof];
    for (int k = 0; k < 8; ++k) {
      F.P.col.push_back(16 * a + 8 * s + k);
      F.P.val.push_back(F.Pblk[(((size_t)a * 2 + s) * F.rows_per + r) * 8 + k]);
    }
    F.P.ptr[dof + 1] = (int)F.P.col.size();
  }
  F.PH = csr_adjoint(F.P);
}

// Least squares fit (eq. LSfuncrowi) per aggregate and spin with k test
// vectors V (column-major, V[j*n + dof]).  For k <= 8 the columns of P_{a,s}
// are the Gram-Schmidt basis of the test vectors restricted to the block
// (classical Gram-Schmidt applied twice, positive R_jj), in test-vector order.
// Columns whose remaining norm vanishes are left zero.
void fit_P(Level& F, bool fine, const std::vector<cplx>& V, int k) {
  AggMap M = aggregate_map(F, fine);
  int n = F.A.nr, na = F.cx * F.cy, R = F.rows_per;
  F.Pblk.assign((size_t)na * 2 * R * 8, 0.0);
  // gather blocks
  std::vector<cplx> blk((size_t)na * 2 * R * k, 0.0);  // [a][s][row][j]
  for (int j = 0; j < k; ++j)
    for (int dof = 0; dof < n; ++dof)
      blk[(((size_t)M.agg[dof] * 2 + M.spin[dof]) * R + M.row[dof]) * k + j] = V[(size_t)j * n + dof];
  int ncol = std::min(k, 8);
  for (int a = 0; a < na; ++a)
    for (int s = 0; s < 2; ++s) {
      cplx* B = &blk[(((size_t)a * 2 + s) * R) * k];
      cplx* Q = &F.Pblk[(((size_t)a * 2 + s) * R) * 8];
      for (int j = 0; j < ncol; ++j) {
        std::vector<cplx> w(R);
        for (int i = 0; i < R; ++i) w[i] = B[i * k + j];
        for (int pass = 0; pass < 2; ++pass) {
          std::vector<cplx> h(j, 0.0);
          for (int q = 0; q < j; ++q)
            for (int i = 0; i < R; ++i) h[q] += std::conj(Q[i * 8 + q]) * w[i];
          for (int q = 0; q < j; ++q)
            for (int i = 0; i < R; ++i) w[i] -= Q[i * 8 + q] * h[q];
        }
        double nrm = 0.0;
        for (int i = 0; i < R; ++i) nrm += std::norm(w[i]);
        nrm = std::sqrt(nrm);
        if (nrm > 0.0)
          for (int i = 0; i < R; ++i) Q[i * 8 + j] = w[i] / nrm;
      }
    }
  build_P_csr(F, fine);
}

// dense LU with partial pivoting (max |.|, lowest row on ties)
void lu_factor(Level& L) {
  int n = L.A.nr;
  L.LU.assign((size_t)n * n, 0.0);
  for (int r = 0; r < n; ++r)
    for (int p = L.A.ptr[r]; p < L.A.ptr[r + 1]; ++p) L.LU[(size_t)r * n + L.A.col[p]] += L.A.val[p];
  L.piv.resize(n); L.singular = false;
  cplx* a = L.LU.data();
  for (int k = 0; k < n; ++k) {
    int p = k; double best = std::abs(a[(size_t)k * n + k]);
    for (int i = k + 1; i < n; ++i) {
      double v = std::abs(a[(size_t)i * n + k]);
      if (v > best) { best = v; p = i; }
    }
    L.piv[k] = p;
    if (best == 0.0) { L.singular = true; continue; }
    if (p != k)
      for (int j = 0; j < n; ++j) std::swap(a[(size_t)k * n + j], a[(size_t)p * n + j]);
    cplx piv = a[(size_t)k * n + k];
#pragma omp parallel for schedule(static)
    for (int i = k + 1; i < n; ++i) {
      cplx l = a[(size_t)i * n + k] / piv;
      a[(size_t)i * n + k] = l;
      for (int j = k + 1; j < n; ++j) a[(size_t)i * n + j] -= l * a[(size_t)k * n + j];
    }
  }
}

void lu_solve(const Level& L, const cplx* b, cplx* x) {
  int n = L.A.nr;
  std::vector<cplx> y(b, b + n);
  for (int k = 0; k < n; ++k) std::swap(y[k], y[L.piv[k]]);
  const cplx* a = L.LU.data();
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j) y[i] -= a[(size_t)i * n + j] * y[j];
  for (int i = n - 1; i >= 0; --i) {
    for (int j = i + 1; j < n; ++j) y[i] -= a[(size_t)i * n + j] * y[j];
    y[i] /= a[(size_t)i * n + i];
  }
  for (int i = 0; i < n; ++i) x[i] = y[i];
}

// ---------------------------------------------------------------------------
// Hierarchy, cycle, setup, FGMRES.
// ---------------------------------------------------------------------------
struct Hier {
  Problem prob;
  std::vector<Level> lv;
  int pre = 4, post = 4, cycle = 0;  // cycle: 0 V, 1 W, 2 K
  int n_tv = 8, sweeps = 20, adapt = 1;
  std::vector<cplx> tv;  // level-1 test vectors after setup, [k][n1]
  // bootstrap eigensolver: eigenvector approximations V^e on level 1 and their Ritz values
  std::vector<cplx> tve;
  std::vector<double> lam;
};

double vnorm(const cplx* v, int n) {
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += std::norm(v[i]);
  return std::sqrt(s);
}

void coarsen_level(Hier& h, int l);
void mg_cycle(Hier& h, int l, const cplx* b, cplx* x);

// <u, v> = sum_i conj(u_i) v_i
cplx vdot(const cplx* u, const cplx* v, int n) {
  cplx s = 0.0;
  for (int i = 0; i < n; ++i) s += std::conj(u[i]) * v[i];
  return s;
}

// K-cycle coarse visit: two steps of flexible GCR on A_c x = r0 from x = 0,
// each step preconditioned by one cycle from level c.
//   z1 = M r0, w1 = A z1, a1 = <w1, r0> / <w1, w1>, x = a1 z1, r1 = r0 - a1 w1,
//   z2 = M r1, w2 = A z2, beta = <w1, w2> / <w1, w1>, w2 -= beta w1, z2 -= beta z1,
//   a2 = <w2, r1> / <w2, w2>, x += a2 z2.
// A step whose <w, w> vanishes adds nothing.
void kcycle_visit(Hier& h, int c, const cplx* r0, cplx* x) {
  const CSR& A = h.lv[c].A;
  int n = A.nr;
  std::vector<cplx> z1(n, 0.0), w1(n), r1(n), z2(n, 0.0), w2(n);
  std::fill(x, x + n, cplx(0.0));
  mg_cycle(h, c, r0, z1.data());
  csr_mv(A, z1.data(), w1.data());
  double rho1 = vdot(w1.data(), w1.data(), n).real();
  if (rho1 == 0.0) return;
  cplx a1 = vdot(w1.data(), r0, n) / rho1;
  for (int i = 0; i < n; ++i) {
    x[i] = a1 * z1[i];
    r1[i] = r0[i] - a1 * w1[i];
  }
  mg_cycle(h, c, r1.data(), z2.data());
  csr_mv(A, z2.data(), w2.data());
  cplx beta = vdot(w1.data(), w2.data(), n) / rho1;
  for (int i = 0; i < n; ++i) {
    w2[i] -= beta * w1[i];
    z2[i] -= beta * z1[i];
  }
  double rho2 = vdot(w2.data(), w2.data(), n).real();
  if (rho2 == 0.0) return;
  cplx a2 = vdot(w2.data(), r1.data(), n) / rho2;
  for (int i = 0; i < n; ++i) x[i] += a2 * z2[i];
}

// multigrid cycle on level l: x (in/out, initial guess) for A_l x = b
void mg_cycle(Hier& h, int l, const cplx* b, cplx* x) {
  Level& L = h.lv[l];
  int n = L.A.nr;
  if (l == (int)h.lv.size() - 1) { lu_solve(L, b, x); return; }
  for (int i = 0; i < h.pre; ++i) kaczmarz_sweep(L, x, b);
  std::vector<cplx> r(n);
  csr_mv(L.A, x, r.data());
  for (int i = 0; i < n; ++i) r[i] = b[i] - r[i];
  int nc = h.lv[l + 1].A.nr;
  std::vector<cplx> bc(nc), xc(nc, 0.0);
  csr_mv(L.PH, r.data(), bc.data());
  bool coarsest_next = (l + 1 == (int)h.lv.size() - 1);
  if (h.cycle == 2 && !coarsest_next) {
    kcycle_visit(h, l + 1, bc.data(), xc.data());
  } else {
    int gamma = (h.cycle == 1) ? 2 : 1;
    for (int g = 0; g < gamma; ++g) {
      mg_cycle(h, l + 1, bc.data(), xc.data());
      if (coarsest_next) break;  // exact solve: a second visit changes nothing
    }
  }
  std::vector<cplx> e(n);
  csr_mv(L.P, xc.data(), e.data());
  for (int i = 0; i < n; ++i) x[i] += e[i];
  for (int i = 0; i < h.post; ++i) kaczmarz_sweep(L, x, b);
}

// level l -> l+1: Galerkin operator, ordering, and (if coarsest) LU
void coarsen_level(Hier& h, int l) {
  Level& F = h.lv[l];
  Level& C = h.lv[l + 1];
  C.A = csr_mul(F.PH, csr_mul(F.A, F.P));
  level_norms_and_order(C, false, h.prob.N);
  if (l + 1 == (int)h.lv.size() - 1) lu_factor(C);
}

// relax k vectors with `sweeps` Kaczmarz sweeps on A_l v = 0, then unit-normalise
void relax_tvs(Hier& h, int l, std::vector<cplx>& V, int k) {
  Level& L = h.lv[l]; int n = L.A.nr;
  for (int j = 0; j < k; ++j) {
    cplx* v = &V[(size_t)j * n];
    for (int s = 0; s < h.sweeps; ++s) kaczmarz_sweep(L, v, nullptr);
    double nv = vnorm(v, n);
    if (nv > 0) for (int i = 0; i < n; ++i) v[i] /= nv;
  }
}

// one relax-fit-coarsen pass from level-1 vectors V1
void setup_pass(Hier& h, std::vector<cplx> V) {
  int k = h.n_tv;
  for (int l = 0; l + 1 < (int)h.lv.size(); ++l) {
    relax_tvs(h, l, V, k);
    if (l == 0) h.tv = V;
    fit_P(h.lv[l], l == 0, V, k);
    coarsen_level(h, l);
    int nc = h.lv[l + 1].A.nr, n = h.lv[l].A.nr;
    std::vector<cplx> Vc((size_t)k * nc);
    for (int j = 0; j < k; ++j) csr_mv(h.lv[l].PH, &V[(size_t)j * n], &Vc[(size_t)j * nc]);
    V.swap(Vc);
  }
}

// ---------------------------------------------------------------------------
// Bootstrap multigrid eigensolver (Sec. 3.4, Theorem 1 of Sec. 3.5).  With
// R = (Gamma_5 P)^H and P orthonormal per aggregate, Q_l = T_l = P_l^H P_l = I,
// and the singular-triplet systems (eq. SVDRnP1-4) reduce to the Hermitian
// eigenproblem Z_l v = lambda v with Z_l = Gamma_5 D_l (Theorem 1 (i), (ii));
// singular values are |lambda| (Theorem 1 (iii)).
// ---------------------------------------------------------------------------

// Gamma_5 on a level: +1 for spin 0, -1 for spin 1 (fine dof 2*site + s,
// coarse dof 16*site + 8*s + k)
double gamma5(const Level& L, int dof) {
  int s = (L.dps == 2) ? (dof & 1) : ((dof % 16) / 8);
  return s == 0 ? 1.0 : -1.0;
}

// eigen-decomposition of the n x n Hermitian H (row-major, destroyed) by cyclic
// Jacobi rotations: w = eigenvalues (unsorted), V = eigenvectors as columns
// (row-major n x n)
void jacobi_eig(int n, std::vector<cplx>& H, std::vector<double>& w, std::vector<cplx>& V) {
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  auto at = [&](int i, int j) -> cplx& { return H[(size_t)i * n + j]; };
  double fro = 0.0;
  for (auto& z : H) fro += std::norm(z);
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        if (i != j) off += std::norm(at(i, j));
    if (off <= 1e-30 * fro || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const cplx hpq = at(p, q);
        const double r = std::abs(hpq);
        if (r == 0.0) continue;
        // phase to a real off-diagonal entry, then the real 2x2 rotation
        const cplx ph = hpq / r;  // e^{i phi}
        const double a = at(p, p).real(), b = at(q, q).real();
        const double tau = (b - a) / (2.0 * r);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (std::abs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), sn = t * c;
        // U = [[c, sn], [-sn e^{-i phi}, c e^{-i phi}]] on columns (p, q)
        const cplx upp = c, upq = sn, uqp = -sn * std::conj(ph), uqq = c * std::conj(ph);
        for (int k = 0; k < n; ++k) {  // H <- H U
          const cplx hkp = at(k, p), hkq = at(k, q);
          at(k, p) = hkp * upp + hkq * uqp;
          at(k, q) = hkp * upq + hkq * uqq;
        }
        for (int k = 0; k < n; ++k) {  // H <- U^H H
          const cplx hpk = at(p, k), hqk = at(q, k);
          at(p, k) = std::conj(upp) * hpk + std::conj(uqp) * hqk;
          at(q, k) = std::conj(upq) * hpk + std::conj(uqq) * hqk;
        }
        at(p, q) = 0.0; at(q, p) = 0.0;
        at(p, p) = at(p, p).real(); at(q, q) = at(q, q).real();
        for (int k = 0; k < n; ++k) {  // V <- V U
          const cplx vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
          V[(size_t)k * n + p] = vkp * upp + vkq * uqp;
          V[(size_t)k * n + q] = vkp * upq + vkq * uqq;
        }
      }
  }
  w.resize(n);
  for (int i = 0; i < n; ++i) w[i] = at(i, i).real();
}

// Ritz value of eq. eqevZ with T = I: <Z v, v> / <v, v>
double ritz_value(const Level& L, const cplx* v) {
  int n = L.A.nr;
  std::vector<cplx> Av(n);
  csr_mv(L.A, v, Av.data());
  cplx num = 0.0;
  double den = 0.0;
  for (int i = 0; i < n; ++i) {
    num += std::conj(v[i]) * gamma5(L, i) * Av[i];
    den += std::norm(v[i]);
  }
  return den > 0 ? num.real() / den : 0.0;
}

// One Kaczmarz sweep (rows in the level's order) on (A - lam Gamma_5) x = 0,
// the row form of Z x = lam x (Theorem 1 (ii)).
void kaczmarz_sweep_shifted(const Level& L, cplx* x, double lam) {
  const CSR& A = L.A;
  for (int r : L.order) {
    const cplx sh = -lam * gamma5(L, r);  // added to the diagonal entry of row r
    bool has_diag = false;
    double nu = 0.0;
    cplx res = 0.0;
    for (int p = A.ptr[r]; p < A.ptr[r + 1]; ++p) {
      cplx a = A.val[p];
      if (A.col[p] == r) { a += sh; has_diag = true; }
      nu += std::norm(a);
      res -= a * x[A.col[p]];
    }
    if (!has_diag) { nu += std::norm(sh); res -= sh * x[r]; }
    if (nu == 0.0) continue;
    const cplx alpha = res / nu;
    for (int p = A.ptr[r]; p < A.ptr[r + 1]; ++p) {
      cplx a = A.val[p];
      if (A.col[p] == r) a += sh;
      x[A.col[p]] += alpha * std::conj(a);
    }
    if (!has_diag) x[r] += alpha * std::conj(sh);
  }
}

// the ke eigenpairs of Z_L = Gamma_5 A_L with the smallest |lambda| (ties by
// index), eigenvectors of unit norm: vals[ke], vecs[ke][n]
void coarsest_eigs(const Level& L, int ke, std::vector<double>& vals, std::vector<cplx>& vecs) {
  int n = L.A.nr;
  std::vector<cplx> Z((size_t)n * n, 0.0);
  for (int r = 0; r < n; ++r)
    for (int p = L.A.ptr[r]; p < L.A.ptr[r + 1]; ++p) Z[(size_t)r * n + L.A.col[p]] += gamma5(L, r) * L.A.val[p];
  std::vector<double> w;
  std::vector<cplx> V;
  jacobi_eig(n, Z, w, V);
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return std::abs(w[a]) < std::abs(w[b]); });
  vals.resize(ke);
  vecs.assign((size_t)ke * n, 0.0);
  for (int k = 0; k < ke && k < n; ++k) {
    vals[k] = w[idx[k]];
    for (int i = 0; i < n; ++i) vecs[(size_t)k * n + i] = V[(size_t)i * n + idx[k]];
  }
}

// Least squares fit (eq. LSfuncrowi) with k > 8 test vectors and 8 columns per
// aggregate and spin: the columns of P_{a,s} span the best rank-8 fit of the
// block of test vectors (unit weights), i.e. the 8 dominant eigenvectors of
// B B^H; the basis is fixed as the Gram-Schmidt basis (applied twice, R_jj > 0)
// of the projections of the first 8 test vectors onto that space.  For k <= 8
// this is fit_P.
void fit_P_ls(Level& F, bool fine, const std::vector<cplx>& V, int k) {
  if (k <= 8) { fit_P(F, fine, V, k); return; }
  AggMap M = aggregate_map(F, fine);
  int n = F.A.nr, na = F.cx * F.cy, R = F.rows_per;
  F.Pblk.assign((size_t)na * 2 * R * 8, 0.0);
  std::vector<cplx> blk((size_t)na * 2 * R * k, 0.0);  // [a][s][row][j]
  for (int j = 0; j < k; ++j)
    for (int dof = 0; dof < n; ++dof)
      blk[(((size_t)M.agg[dof] * 2 + M.spin[dof]) * R + M.row[dof]) * k + j] = V[(size_t)j * n + dof];
  for (int a = 0; a < na; ++a)
    for (int s = 0; s < 2; ++s) {
      const cplx* B = &blk[(((size_t)a * 2 + s) * R) * k];
      std::vector<cplx> G((size_t)R * R, 0.0);
      for (int i = 0; i < R; ++i)
        for (int i2 = 0; i2 < R; ++i2)
          for (int j = 0; j < k; ++j) G[(size_t)i * R + i2] += B[i * k + j] * std::conj(B[i2 * k + j]);
      std::vector<double> w;
      std::vector<cplx> E;
      jacobi_eig(R, G, w, E);
      std::vector<int> idx(R);
      for (int i = 0; i < R; ++i) idx[i] = i;
      std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return w[x] > w[y]; });
      cplx* Q = &F.Pblk[(((size_t)a * 2 + s) * R) * 8];
      for (int j = 0; j < 8; ++j) {
        // projection of test vector j onto the span of the 8 dominant eigenvectors
        std::vector<cplx> wv(R, 0.0);
        for (int e = 0; e < 8; ++e) {
          cplx c = 0.0;
          for (int i = 0; i < R; ++i) c += std::conj(E[(size_t)i * R + idx[e]]) * B[i * k + j];
          for (int i = 0; i < R; ++i) wv[i] += E[(size_t)i * R + idx[e]] * c;
        }
        for (int pass = 0; pass < 2; ++pass) {
          std::vector<cplx> hq(j, 0.0);
          for (int q = 0; q < j; ++q)
            for (int i = 0; i < R; ++i) hq[q] += std::conj(Q[i * 8 + q]) * wv[i];
          for (int q = 0; q < j; ++q)
            for (int i = 0; i < R; ++i) wv[i] -= Q[i * 8 + q] * hq[q];
        }
        double nrm = 0.0;
        for (int i = 0; i < R; ++i) nrm += std::norm(wv[i]);
        nrm = std::sqrt(nrm);
        if (nrm > 0.0)
          for (int i = 0; i < R; ++i) Q[i * 8 + j] = wv[i] / nrm;
      }
    }
  build_P_csr(F, fine);
}

// ---------------------------------------------------------------------------
// Bootstrap setup cycles (Sec. 3.4, its setup-cycle figure, Sec. 4.1 / 4.2).
// Per level: relaxation test vectors V^r (k_r) and eigenvector approximations
// V^e (k_e) with their Ritz values.  Node kinds of the setup-cycle figure:
//   arrive (first visit of the first cycle): relax V^r on Z v = 0, compute P;
//   arrive (later): relax V^r on Z v = 0 and V^e on Z v = lambda T v, recompute P;
//   coarsest: the k_e eigenpairs of Z_L with the smallest |lambda| replace V^e;
//   after the last visit below: relax V^e on Z v = lambda T v.
// Computing P on level l also rebuilds level l+1 (Galerkin) and restricts
// both sets of test vectors to it; coming back up, V^e_l = P_l V^e_{l+1}.
// ---------------------------------------------------------------------------
struct BootSets {
  std::vector<std::vector<cplx>> Vr, Ve;  // per level, [k][n_l]
  std::vector<double> lam;                // Ritz values of V^e
  int kr = 8, ke = 0;
  bool have_e = false;
};

void unit_normalise(cplx* v, int n) {
  double nv = vnorm(v, n);
  if (nv > 0) for (int i = 0; i < n; ++i) v[i] /= nv;
}

void boot_relax_r(Hier& h, int l, BootSets& B, int nu) {
  Level& L = h.lv[l]; int n = L.A.nr;
  for (int j = 0; j < B.kr; ++j) {
    cplx* v = &B.Vr[l][(size_t)j * n];
    for (int s = 0; s < nu; ++s) kaczmarz_sweep(L, v, nullptr);
    unit_normalise(v, n);
  }
}

// Kaczmarz on (A - lambda Gamma_5) v = 0 with the Ritz value updated after every sweep (eq. eqevZ)
void boot_relax_e(Hier& h, int l, BootSets& B, int nu) {
  if (!B.have_e) return;
  Level& L = h.lv[l]; int n = L.A.nr;
  for (int j = 0; j < B.ke; ++j) {
    cplx* v = &B.Ve[l][(size_t)j * n];
    for (int s = 0; s < nu; ++s) {
      kaczmarz_sweep_shifted(L, v, B.lam[j]);
      B.lam[j] = ritz_value(L, v);
    }
    unit_normalise(v, n);
  }
}

void boot_fit(Hier& h, int l, BootSets& B) {
  Level& L = h.lv[l]; int n = L.A.nr;
  int k = B.kr + (B.have_e ? B.ke : 0);
  std::vector<cplx> V((size_t)k * n);
  std::copy(B.Vr[l].begin(), B.Vr[l].end(), V.begin());
  if (B.have_e) std::copy(B.Ve[l].begin(), B.Ve[l].end(), V.begin() + (size_t)B.kr * n);
  fit_P_ls(L, l == 0, V, k);
  coarsen_level(h, l);
  int nc = h.lv[l + 1].A.nr;
  B.Vr[l + 1].assign((size_t)B.kr * nc, 0.0);
  for (int j = 0; j < B.kr; ++j) csr_mv(L.PH, &B.Vr[l][(size_t)j * n], &B.Vr[l + 1][(size_t)j * nc]);
  if (B.have_e) {
    B.Ve[l + 1].assign((size_t)B.ke * nc, 0.0);
    for (int j = 0; j < B.ke; ++j) csr_mv(L.PH, &B.Ve[l][(size_t)j * n], &B.Ve[l + 1][(size_t)j * nc]);
  }
}

void boot_interp_e(Hier& h, int l, BootSets& B) {
  Level& L = h.lv[l]; int n = L.A.nr, nc = h.lv[l + 1].A.nr;
  B.Ve[l].assign((size_t)B.ke * n, 0.0);
  for (int j = 0; j < B.ke; ++j) csr_mv(L.P, &B.Ve[l + 1][(size_t)j * nc], &B.Ve[l][(size_t)j * n]);
}

void boot_coarsest(Hier& h, BootSets& B, int ke) {
  int Lc = (int)h.lv.size() - 1;
  coarsest_eigs(h.lv[Lc], ke, B.lam, B.Ve[Lc]);
  B.ke = ke;
  B.have_e = true;
}

void boot_arrive(Hier& h, int l, BootSets& B, int nu, bool first) {
  boot_relax_r(h, l, B, nu);
  if (!first) boot_relax_e(h, l, B, nu);
  boot_fit(h, l, B);
}

// visit of level l >= 1 inside a setup cycle; nu[l] sweeps per node, gamma visits below
void boot_visit(Hier& h, int l, BootSets& B, const std::vector<int>& nu, bool first, int gamma, int ke) {
  int Lc = (int)h.lv.size() - 1;
  boot_arrive(h, l, B, nu[l], first);
  for (int g = 0; g < gamma; ++g) {
    if (l + 1 == Lc) boot_coarsest(h, B, ke);
    else boot_visit(h, l + 1, B, nu, first && g == 0, gamma, ke);
    boot_interp_e(h, l, B);
    if (g < gamma - 1) boot_arrive(h, l, B, nu[l], false);
    else boot_relax_e(h, l, B, nu[l]);
  }
}

// one setup cycle from the finest level (visited once per cycle)
void boot_cycle(Hier& h, BootSets& B, const std::vector<int>& nu, bool first, int gamma, int ke) {
  int Lc = (int)h.lv.size() - 1;
  boot_arrive(h, 0, B, nu[0], first);
  if (Lc == 1) boot_coarsest(h, B, ke);
  else boot_visit(h, 1, B, nu, first, gamma, ke);
  boot_interp_e(h, 0, B);
  boot_relax_e(h, 0, B, nu[0]);
}

// the schedule of Sec. 4.1 (mode 1: W(nu1,nu1) setup cycle, adaptive step, W(nu2,nu2))
// or Sec. 4.2 (mode 2: super-V, mu 2^l sweeps on level l, mu = nu1 then nu2)
void boot_setup(Hier& h, const std::vector<cplx>& V0, int mode, int ke, int nu1, int nu2, int adapt_cycles) {
  int L = (int)h.lv.size();
  BootSets B;
  B.kr = h.n_tv;
  B.Vr.resize(L); B.Ve.resize(L);
  B.Vr[0] = V0;
  int gamma = (mode == 1) ? 2 : 1;
  auto sweeps = [&](int mu) {
    std::vector<int> nu(L);
    for (int l = 0; l < L; ++l) nu[l] = (mode == 1) ? mu : mu * (1 << l);
    return nu;
  };
  boot_cycle(h, B, sweeps(nu1), true, gamma, ke);
  // adaptive step: cycles of the current solver on Dhat v = 0 for the
  // eigenvector approximation with the smallest |Ritz value|
  int n1 = h.lv[0].A.nr;
  int kmin = 0;
  for (int j = 1; j < B.ke; ++j)
    if (std::abs(B.lam[j]) < std::abs(B.lam[kmin])) kmin = j;
  std::vector<cplx> zero(n1, 0.0);
  cplx* v = &B.Ve[0][(size_t)kmin * n1];
  for (int c = 0; c < adapt_cycles; ++c) mg_cycle(h, 0, zero.data(), v);
  unit_normalise(v, n1);
  B.lam[kmin] = ritz_value(h.lv[0], v);
  boot_cycle(h, B, sweeps(nu2), false, gamma, ke);
  h.tv = B.Vr[0];
  h.tve = B.Ve[0];
  h.lam = B.lam;
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), written from its definition.
void philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// complex Gaussian with Re, Im iid N(0, 1/2) for level-1 dof `dof` of test
// vector `j` (Box-Muller on two 53-bit uniforms in (0,1)).
cplx tv_entry(uint64_t seed, int j, int dof) {
  uint32_t ctr[4] = {(uint32_t)dof, (uint32_t)j, 0u, 0u};
  uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
  uint32_t r[4];
  philox4x32_10(ctr, key, r);
  const double two53 = 9007199254740992.0;
  double u1 = ((double)(r[0] >> 5) * 67108864.0 + (double)(r[1] >> 6) + 0.5) / two53;
  double u2 = ((double)(r[2] >> 5) * 67108864.0 + (double)(r[3] >> 6) + 0.5) / two53;
  double rho = std::sqrt(-2.0 * std::log(u1));
  double th = 2.0 * M_PI * u2;
  return cplx(rho * std::cos(th), rho * std::sin(th)) / std::sqrt(2.0);
}

}  // namespace

// ===========================================================================
// C interface (host pointers; complex numbers are interleaved (re, im) doubles)
// ===========================================================================
extern "C" {

int oracle_version(void) { return 1; }

void oracle_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
  philox4x32_10(ctr, key, out);
}

// k test vectors on level 1 (reduced layout), out[j][dof], dof = 2*e + s
void oracle_gaussian_tv(int N, int k, uint64_t seed, double* out) {
  int n = N * N;
  cplx* o = (cplx*)out;
  for (int j = 0; j < k; ++j)
    for (int d = 0; d < n; ++d) o[(size_t)j * n + d] = tv_entry(seed, j, d);
}

// D psi for the full lattice, D = (m+2) I - H
void oracle_wilson_apply(int N, const double* U, double m, const double* in, double* out) {
  CSR H = build_hop(N, (const cplx*)U);
  int n = 2 * N * N;
  std::vector<cplx> t(n);
  csr_mv(H, (const cplx*)in, t.data());
  const cplx* x = (const cplx*)in; cplx* y = (cplx*)out;
  for (int i = 0; i < n; ++i) y[i] = (m + 2.0) * x[i] - t[i];
}

// dense D (row-major, 2N^2 x 2N^2), small N only
void oracle_wilson_dense(int N, const double* U, double m, double* out) {
  CSR H = build_hop(N, (const cplx*)U);
  int n = 2 * N * N;
  cplx* D = (cplx*)out;
  std::fill(D, D + (size_t)n * n, cplx(0.0));
  for (int r = 0; r < n; ++r) {
    D[(size_t)r * n + r] += m + 2.0;
    for (int p = H.ptr[r]; p < H.ptr[r + 1]; ++p) D[(size_t)r * n + H.col[p]] -= H.val[p];
  }
}

// CSR export of the full Wilson operator D (for spectral calibration)
int oracle_wilson_csr_nnz(int N, const double* U) { return (int)build_hop(N, (const cplx*)U).col.size() + 2 * N * N; }
void oracle_wilson_csr(int N, const double* U, double m, int* ptr, int* col, double* val) {
  CSR H = build_hop(N, (const cplx*)U);
  int n = 2 * N * N, q = 0;
  ptr[0] = 0;
  for (int r = 0; r < n; ++r) {
    col[q] = r; ((cplx*)val)[q] = m + 2.0; ++q;
    for (int p = H.ptr[r]; p < H.ptr[r + 1]; ++p) { col[q] = H.col[p]; ((cplx*)val)[q] = -H.val[p]; ++q; }
    ptr[r + 1] = q;
  }
}

// dense Dhat (row-major, N^2 x N^2), small N only
void oracle_dhat_dense(int N, const double* U, double m, double* out) {
  Problem P; build_problem(P, N, U, m);
  int n = N * N;
  cplx* D = (cplx*)out;
  std::fill(D, D + (size_t)n * n, cplx(0.0));
  for (int r = 0; r < n; ++r)
    for (int p = P.Dhat.ptr[r]; p < P.Dhat.ptr[r + 1]; ++p) D[(size_t)r * n + P.Dhat.col[p]] += P.Dhat.val[p];
}

// y = Dhat x for nrhs reduced vectors [nrhs][N^2]
void oracle_dhat_apply(int N, const double* U, double m, const double* x, double* y, int nrhs) {
  Problem P; build_problem(P, N, U, m);
  int n = N * N;
  for (int j = 0; j < nrhs; ++j) csr_mv(P.Dhat, (const cplx*)x + (size_t)j * n, (cplx*)y + (size_t)j * n);
}

// bhat = b_e/c + c^-2 H_eo b_o  (full-lattice b, reduced bhat)
void oracle_eo_reduce(int N, const double* U, double m, const double* b, double* bhat, int nrhs) {
  Problem P; build_problem(P, N, U, m);
  int half = N / 2, n = N * N;
  for (int j = 0; j < nrhs; ++j) {
    const cplx* bf = (const cplx*)b + (size_t)j * 2 * n;
    cplx* out = (cplx*)bhat + (size_t)j * n;
    std::vector<cplx> be(n), bo(n), t(n);
    for (int y = 0; y < N; ++y)
      for (int xh = 0; xh < half; ++xh)
        for (int s = 0; s < 2; ++s) {
          be[2 * (y * half + xh) + s] = bf[2 * (y * N + even_site_x(xh, y)) + s];
          bo[2 * (y * half + xh) + s] = bf[2 * (y * N + odd_site_x(xh, y)) + s];
        }
    csr_mv(P.Heo, bo.data(), t.data());
    for (int i = 0; i < n; ++i) out[i] = be[i] / P.c + t[i] / (P.c * P.c);
  }
}

// full x from x_e:  x_o = b_o/c + c^-1 H_oe x_e
void oracle_eo_reconstruct(int N, const double* U, double m, const double* b, const double* xe, double* x, int nrhs) {
  Problem P; build_problem(P, N, U, m);
  int half = N / 2, n = N * N;
  for (int j = 0; j < nrhs; ++j) {
    const cplx* bf = (const cplx*)b + (size_t)j * 2 * n;
    const cplx* xr = (const cplx*)xe + (size_t)j * n;
    cplx* xf = (cplx*)x + (size_t)j * 2 * n;
    std::vector<cplx> t(n);
    csr_mv(P.Hoe, xr, t.data());
    for (int y = 0; y < N; ++y)
      for (int xh = 0; xh < half; ++xh)
        for (int s = 0; s < 2; ++s) {
          int r = 2 * (y * half + xh) + s;
          xf[2 * (y * N + even_site_x(xh, y)) + s] = xr[r];
          xf[2 * (y * N + odd_site_x(xh, y)) + s] = bf[2 * (y * N + odd_site_x(xh, y)) + s] / P.c + t[r] / P.c;
        }
  }
}

// `sweeps` fine Kaczmarz sweeps on Dhat x = b (b may be null for b = 0), in place
void oracle_kaczmarz_fine(int N, const double* U, double m, double* x, const double* b, int sweeps, int nrhs) {
  Problem P; build_problem(P, N, U, m);
  Level L; L.ex = N / 2; L.ey = N; L.dps = 2; L.A = P.Dhat;
  level_norms_and_order(L, true, N);
  int n = N * N;
  for (int j = 0; j < nrhs; ++j)
    for (int s = 0; s < sweeps; ++s)
      kaczmarz_sweep(L, (cplx*)x + (size_t)j * n, b ? (const cplx*)b + (size_t)j * n : nullptr);
}

// the fine colour of even site (x, y) and the coarse colour map (for tests)
int oracle_fine_colour(int x, int y) { return fine_colour(x, y); }
int oracle_coarse_colour(int ax, int ay, int ex, int ey) { return coarse_colour(ax, ay, ex, ey); }
int oracle_coarse_ncolours(int ex, int ey) { return coarse_ncolours(ex, ey); }

// ---------------------------------------------------------------------------
// hierarchy interface
// ---------------------------------------------------------------------------
void* oracle_setup(int N, const double* U, double m, int n_levels, int max_coarse, int n_tv,
                   int sweeps, int adapt, int pre, int post, int cycle, uint64_t seed,
                   const double* init_tv) {
  if (N % 8 != 0 || N < 16 || n_tv < 1 || n_tv > 8) return nullptr;
  Hier* h = new Hier();
  build_problem(h->prob, N, U, m);
  h->pre = pre; h->post = post; h->cycle = cycle; h->n_tv = n_tv; h->sweeps = sweeps; h->adapt = adapt;
  // level shapes
  std::vector<std::pair<int, int>> ext;
  ext.push_back({N / 2, N});
  int ex = N / 8, ey = N / 4;
  ext.push_back({ex, ey});
  while (true) {
    int L = (int)ext.size();
    if (n_levels > 0 && L >= n_levels) break;
    if (n_levels <= 0 && ex * ey * 16 <= max_coarse) break;
    if (ex % 2 || ey % 2 || ex < 4 || ey < 4) break;
    ex /= 2; ey /= 2;
    ext.push_back({ex, ey});
  }
  h->lv.resize(ext.size());
  for (size_t l = 0; l < ext.size(); ++l) {
    h->lv[l].ex = ext[l].first; h->lv[l].ey = ext[l].second; h->lv[l].dps = (l == 0) ? 2 : 16;
    if (l + 1 < ext.size()) {
      h->lv[l].cx = ext[l + 1].first; h->lv[l].cy = ext[l + 1].second;
      h->lv[l].ax = (l == 0) ? 4 : 2; h->lv[l].ay = (l == 0) ? 4 : 2;
      h->lv[l].rows_per = (l == 0) ? 16 : 32;
    }
  }
  h->lv[0].A = h->prob.Dhat;
  level_norms_and_order(h->lv[0], true, N);
  int n1 = N * N;
  std::vector<cplx> V((size_t)n_tv * n1);
  if (init_tv) std::copy((const cplx*)init_tv, (const cplx*)init_tv + V.size(), V.begin());
  else for (int j = 0; j < n_tv; ++j) for (int d = 0; d < n1; ++d) V[(size_t)j * n1 + d] = tv_entry(seed, j, d);
  if (adapt < 0) return h;  // shapes and operator only (the bootstrap setup builds the rest)
  setup_pass(*h, V);
  for (int a = 0; a < adapt; ++a) {
    // adaptive step: two cycles of the current hierarchy on Dhat v = 0 per test vector
    std::vector<cplx> W = h->tv;
    std::vector<cplx> zero(n1, 0.0);
    for (int j = 0; j < n_tv; ++j) {
      cplx* v = &W[(size_t)j * n1];
      for (int c = 0; c < 2; ++c) mg_cycle(*h, 0, zero.data(), v);
      double nv = vnorm(v, n1);
      if (nv > 0) for (int i = 0; i < n1; ++i) v[i] /= nv;
    }
    setup_pass(*h, W);
  }
  return h;
}

void oracle_free(void* hp) { delete (Hier*)hp; }

// Hierarchy by the bootstrap setup cycles (mode 1: W, mode 2: super-V; see
// boot_setup); the other arguments as oracle_setup.
void* oracle_setup_boot(int N, const double* U, double m, int n_levels, int max_coarse, int pre, int post,
                        int cycle, uint64_t seed, const double* init_tv, int mode, int ke, int nu1, int nu2,
                        int adapt_cycles) {
  if (mode != 1 && mode != 2) return nullptr;
  // shapes, operator and random test vectors as in oracle_setup, without its setup passes
  Hier* h = (Hier*)oracle_setup(N, U, m, n_levels, max_coarse, 8, 0, -1, pre, post, cycle, seed, init_tv);
  if (!h || h->lv.size() < 2) return h;
  int n1 = N * N;
  std::vector<cplx> V((size_t)8 * n1);
  if (init_tv) std::copy((const cplx*)init_tv, (const cplx*)init_tv + V.size(), V.begin());
  else for (int j = 0; j < 8; ++j) for (int d = 0; d < n1; ++d) V[(size_t)j * n1 + d] = tv_entry(seed, j, d);
  boot_setup(*h, V, mode, ke, nu1, nu2, adapt_cycles);
  return h;
}

// eigen-decomposition of a Hermitian n x n matrix (row-major) by cyclic Jacobi
void oracle_jacobi_eig(int n, const double* H, double* w, double* V) {
  std::vector<cplx> A((const cplx*)H, (const cplx*)H + (size_t)n * n);
  std::vector<double> ww;
  std::vector<cplx> VV;
  jacobi_eig(n, A, ww, VV);
  std::copy(ww.begin(), ww.end(), w);
  std::copy(VV.begin(), VV.end(), (cplx*)V);
}

// Ritz values (eq. eqevZ, T = I) of nrhs level-l vectors
void oracle_ritz(void* hp, int l, const double* x, double* lam, int nrhs) {
  Level& L = ((Hier*)hp)->lv[l];
  for (int j = 0; j < nrhs; ++j) lam[j] = ritz_value(L, (const cplx*)x + (size_t)j * L.A.nr);
}

// one Kaczmarz sweep on (A_l - lam_j Gamma_5) x_j = 0 for nrhs vectors (in place)
void oracle_sweep_shifted(void* hp, int l, double* x, const double* lam, int nrhs) {
  Level& L = ((Hier*)hp)->lv[l];
  for (int j = 0; j < nrhs; ++j) kaczmarz_sweep_shifted(L, (cplx*)x + (size_t)j * L.A.nr, lam[j]);
}

// the ke eigenpairs of Z_L with the smallest |lambda|: vals[ke], vecs[ke][n_L]
void oracle_coarsest_eigs(void* hp, int ke, double* vals, double* vecs) {
  Hier* h = (Hier*)hp;
  std::vector<double> w;
  std::vector<cplx> V;
  coarsest_eigs(h->lv.back(), ke, w, V);
  std::copy(w.begin(), w.end(), vals);
  std::copy(V.begin(), V.end(), (cplx*)vecs);
}

// refit P_l from k level-l test vectors (least squares, rank-8) and rebuild level l+1
void oracle_fit_ls(void* hp, int l, const double* V, int k) {
  Hier* h = (Hier*)hp;
  Level& L = h->lv[l];
  std::vector<cplx> VV((const cplx*)V, (const cplx*)V + (size_t)k * L.A.nr);
  fit_P_ls(L, l == 0, VV, k);
  coarsen_level(*h, l);
}

// eigenvector approximations on level 1 and their Ritz values after a bootstrap setup
int oracle_export_boot(void* hp, double* lam, double* ve) {
  Hier* h = (Hier*)hp;
  int ke = (int)h->lam.size();
  if (lam) std::copy(h->lam.begin(), h->lam.end(), lam);
  if (ve) std::copy(h->tve.begin(), h->tve.end(), (cplx*)ve);
  return ke;
}

int oracle_n_levels(void* hp) { return (int)((Hier*)hp)->lv.size(); }

// level info: extents, dofs per site, operator rows and nnz
void oracle_level_info(void* hp, int l, int* info) {
  Level& L = ((Hier*)hp)->lv[l];
  info[0] = L.ex; info[1] = L.ey; info[2] = L.dps; info[3] = L.A.nr; info[4] = (int)L.A.col.size();
  info[5] = L.singular ? 1 : 0;
}

void oracle_export_op(void* hp, int l, int* ptr, int* col, double* val) {
  Level& L = ((Hier*)hp)->lv[l];
  std::copy(L.A.ptr.begin(), L.A.ptr.end(), ptr);
  std::copy(L.A.col.begin(), L.A.col.end(), col);
  std::copy(L.A.val.begin(), L.A.val.end(), (cplx*)val);
}

// P of level l in aggregate blocks [agg][s][row][8]
void oracle_export_P(void* hp, int l, double* P) {
  Level& L = ((Hier*)hp)->lv[l];
  std::copy(L.Pblk.begin(), L.Pblk.end(), (cplx*)P);
}

void oracle_export_tv(void* hp, double* tv) {
  Hier* h = (Hier*)hp;
  std::copy(h->tv.begin(), h->tv.end(), (cplx*)tv);
}

// replace P of level l (aggregate blocks) and rebuild level l+1 (and the LU if
// coarsest and `factor` is nonzero; else the coarsest level waits for
// oracle_set_coarsest_lu)
void oracle_import_P(void* hp, int l, const double* P, int factor) {
  Hier* h = (Hier*)hp;
  Level& L = h->lv[l];
  L.Pblk.assign((const cplx*)P, (const cplx*)P + (size_t)L.cx * L.cy * 2 * L.rows_per * 8);
  build_P_csr(L, l == 0);
  if (factor) {
    coarsen_level(*h, l);
    return;
  }
  Level& C = h->lv[l + 1];
  C.A = csr_mul(L.PH, csr_mul(L.A, L.P));
  level_norms_and_order(C, false, h->prob.N);
  if (l + 1 == (int)h->lv.size() - 1) { C.LU.clear(); C.piv.clear(); C.singular = true; }
}

// LU factors of the coarsest operator computed elsewhere (row-major n x n, unit
// lower triangle below the diagonal, U on and above it; piv[k]: the row swapped
// with row k at step k, 0-based), for the coarsest solve by substitution
void oracle_set_coarsest_lu(void* hp, const double* LU, const int* piv) {
  Hier* h = (Hier*)hp;
  Level& C = h->lv.back();
  int n = C.A.nr;
  C.LU.assign((const cplx*)LU, (const cplx*)LU + (size_t)n * n);
  C.piv.assign(piv, piv + n);
  C.singular = false;
  for (int i = 0; i < n; ++i)
    if (C.LU[(size_t)i * n + i] == 0.0) C.singular = true;
}

// Stand-alone iteration of the solver on Dhat x = 0 (Sec. 4): x <- x + M(0 - Dhat x)
// with M one cycle (zero initial guess), `iters` times from x (in/out);
// norms[i] = ||x|| after i iterations (norms[0] = ||x0||), so the error
// reduction of iteration i is norms[i] / norms[i-1].
void oracle_stationary(void* hp, double* xio, int iters, double* norms) {
  Hier* h = (Hier*)hp;
  const CSR& A = h->lv[0].A;
  int n = A.nr;
  cplx* x = (cplx*)xio;
  std::vector<cplx> r(n), z(n);
  norms[0] = vnorm(x, n);
  if (h->lv.size() > 1 && h->lv.back().LU.empty()) return;  // coarsest not factored
  for (int it = 0; it < iters; ++it) {
    csr_mv(A, x, r.data());
    for (int i = 0; i < n; ++i) r[i] = -r[i];
    std::fill(z.begin(), z.end(), cplx(0.0));
    mg_cycle(*h, 0, r.data(), z.data());
    for (int i = 0; i < n; ++i) x[i] += z[i];
    norms[it + 1] = vnorm(x, n);
  }
}

// level operations on nrhs vectors: op 0: y = A_l x; 1: x <- one Kaczmarz sweep on
// A_l x = b (in: b, out: x in place); 2: y = P_l^H x (restriction from l to l+1);
// 3: y += P_l x (prolongation from l+1 to l); 4: y = A_L^{-1} x (coarsest);
// 5: y = one multigrid cycle from level l on A_l y = x with zero initial guess.
int oracle_level_op(void* hp, int l, int op, const double* in, double* out, int nrhs) {
  Hier* h = (Hier*)hp;
  Level& L = h->lv[l];
  int n = L.A.nr;
  int nc = (l + 1 < (int)h->lv.size()) ? h->lv[l + 1].A.nr : 0;
  if ((op == 4 || op == 5) && h->lv.back().LU.empty()) return -4;  // coarsest not factored
  for (int j = 0; j < nrhs; ++j) {
    switch (op) {
      case 0: csr_mv(L.A, (const cplx*)in + (size_t)j * n, (cplx*)out + (size_t)j * n); break;
      case 1: kaczmarz_sweep(L, (cplx*)out + (size_t)j * n, (const cplx*)in + (size_t)j * n); break;
      case 2: csr_mv(L.PH, (const cplx*)in + (size_t)j * n, (cplx*)out + (size_t)j * nc); break;
      case 3: {
        std::vector<cplx> e(n);
        csr_mv(L.P, (const cplx*)in + (size_t)j * nc, e.data());
        cplx* o = (cplx*)out + (size_t)j * n;
        for (int i = 0; i < n; ++i) o[i] += e[i];
        break;
      }
      case 4: if (L.singular) return -4; lu_solve(L, (const cplx*)in + (size_t)j * n, (cplx*)out + (size_t)j * n); break;
      case 5: {
        cplx* o = (cplx*)out + (size_t)j * n;
        std::fill(o, o + n, cplx(0.0));
        mg_cycle(*h, l, (const cplx*)in + (size_t)j * n, o);
        break;
      }
      default: return -1;
    }
  }
  return 0;
}

// FGMRES(restart) right-preconditioned by one cycle; x0 = 0; reduced system.
// info: [iters, restarts, relres_reduced, relres_full(unused here), rho_est]
int oracle_solve_reduced(void* hp, const double* bh, double* xo, double tol, int restart, int max_iter,
                         double* info) {
  Hier* h = (Hier*)hp;
  const CSR& A = h->lv[0].A;
  int n = A.nr;
  const cplx* b = (const cplx*)bh;
  cplx* x = (cplx*)xo;
  std::fill(x, x + n, cplx(0.0));
  double bnorm = vnorm(b, n);
  info[0] = 0; info[1] = 0; info[2] = 0; info[3] = 0; info[4] = 0;
  if (!std::isfinite(bnorm)) return -1;
  if (bnorm == 0.0) return 0;
  if (h->lv.back().LU.empty()) return -4;  // coarsest not factored
  std::vector<cplx> r(b, b + n);
  int it = 0, restarts = 0;
  double relres = 1.0;
  int m = restart;
  std::vector<cplx> V((size_t)(m + 1) * n), Z((size_t)m * n), w(n);
  std::vector<cplx> Hm((size_t)(m + 1) * m), cs(m), g(m + 1);
  std::vector<double> cr(m);
  while (true) {
    double beta = vnorm(r.data(), n);
    relres = beta / bnorm;
    if (relres <= tol) break;
    if (it >= max_iter) break;
    for (int i = 0; i < n; ++i) V[i] = r[i] / beta;
    std::fill(g.begin(), g.end(), cplx(0.0)); g[0] = beta;
    std::fill(Hm.begin(), Hm.end(), cplx(0.0));
    int jend = 0;
    for (int j = 0; j < m; ++j) {
      cplx* z = &Z[(size_t)j * n];
      std::fill(z, z + n, cplx(0.0));
      mg_cycle(*h, 0, &V[(size_t)j * n], z);
      csr_mv(A, z, w.data());
      // classical Gram-Schmidt, twice
      for (int pass = 0; pass < 2; ++pass) {
        std::vector<cplx> hh(j + 1, 0.0);
        for (int q = 0; q <= j; ++q) {
          const cplx* vq = &V[(size_t)q * n];
          for (int i = 0; i < n; ++i) hh[q] += std::conj(vq[i]) * w[i];
        }
        for (int q = 0; q <= j; ++q) {
          const cplx* vq = &V[(size_t)q * n];
          for (int i = 0; i < n; ++i) w[i] -= vq[i] * hh[q];
        }
        for (int q = 0; q <= j; ++q) Hm[(size_t)q * m + j] += hh[q];
      }
      double hn = vnorm(w.data(), n);
      Hm[(size_t)(j + 1) * m + j] = hn;
      // previous rotations
      for (int q = 0; q < j; ++q) {
        cplx a = Hm[(size_t)q * m + j], bb = Hm[(size_t)(q + 1) * m + j];
        Hm[(size_t)q * m + j] = cr[q] * a + cs[q] * bb;
        Hm[(size_t)(q + 1) * m + j] = -std::conj(cs[q]) * a + cr[q] * bb;
      }
      // new rotation zeroing H[j+1][j]
      cplx a = Hm[(size_t)j * m + j];
      double bb = hn;
      double t = std::sqrt(std::norm(a) + bb * bb);
      double c; cplx s;
      if (bb == 0.0) { c = 1.0; s = 0.0; }
      else if (std::abs(a) == 0.0) { c = 0.0; s = 1.0; }
      else { c = std::abs(a) / t; s = (a / std::abs(a)) * bb / t; }
      cr[j] = c; cs[j] = s;
      Hm[(size_t)j * m + j] = c * a + s * bb;
      Hm[(size_t)(j + 1) * m + j] = 0.0;
      g[j + 1] = -std::conj(s) * g[j];
      g[j] = c * g[j];
      ++it; jend = j + 1;
      if (hn != 0.0) for (int i = 0; i < n; ++i) V[(size_t)(j + 1) * n + i] = w[i] / hn;
      if (std::abs(g[j + 1]) <= tol * bnorm || it >= max_iter || hn == 0.0) break;
    }
    // y = H^{-1} g (upper triangular), x += Z y
    std::vector<cplx> yv(jend);
    for (int i = jend - 1; i >= 0; --i) {
      cplx s = g[i];
      for (int q = i + 1; q < jend; ++q) s -= Hm[(size_t)i * m + q] * yv[q];
      yv[i] = s / Hm[(size_t)i * m + i];
    }
    for (int q = 0; q < jend; ++q)
      for (int i = 0; i < n; ++i) x[i] += Z[(size_t)q * n + i] * yv[q];
    // true residual
    csr_mv(A, x, w.data());
    for (int i = 0; i < n; ++i) r[i] = b[i] - w[i];
    ++restarts;
  }
  info[0] = it; info[1] = restarts > 0 ? restarts - 1 : 0; info[2] = relres;
  info[4] = it > 0 ? std::pow(relres, 1.0 / it) : 0.0;
  return relres <= tol ? 0 : 1;
}

// full solve D psi = b: reduce, FGMRES on Dhat, reconstruct.  info as above plus
// info[3] = ||b - D psi|| / ||b||.
int oracle_solve(void* hp, const double* b, double* x, double tol, int restart, int max_iter, double* info) {
  Hier* h = (Hier*)hp;
  int N = h->prob.N, n = N * N;
  std::vector<cplx> bh(n), xe(n);
  const double* U = (const double*)h->prob.U.data();
  oracle_eo_reduce(N, U, h->prob.m, b, (double*)bh.data(), 1);
  int st = oracle_solve_reduced(hp, (const double*)bh.data(), (double*)xe.data(), tol, restart, max_iter, info);
  oracle_eo_reconstruct(N, U, h->prob.m, b, (const double*)xe.data(), x, 1);
  std::vector<cplx> Dx(2 * n);
  oracle_wilson_apply(N, U, h->prob.m, x, (double*)Dx.data());
  double rn = 0, bn = 0;
  for (int i = 0; i < 2 * n; ++i) { rn += std::norm(((const cplx*)b)[i] - Dx[i]); bn += std::norm(((const cplx*)b)[i]); }
  info[3] = bn > 0 ? std::sqrt(rn / bn) : 0.0;
  return st;
}

}  // extern "C"
