/*
 * bamg.h -- C ABI of libbamg: bootstrap algebraic multigrid (Brannick & Kahl,
 * arXiv:1308.5992) for the odd-even reduced 2D Wilson-Dirac system on AMD
 * MI355X (gfx950), as a preconditioner of a flexible GMRES in FP64.
 *
 * The problem (Sec. 1, eq. dirac; Sec. 2, eq. wilson): solve D psi = b on an
 * N x N periodic lattice with U(1) links, two spin components per site and
 * D = (m + 2) I - H, where H is the Wilson hopping term of eq. (wilson).
 * The library solves the odd-even reduced system of Sec. 3.2 / Sec. 4,
 * Dhat x_e = bhat with c = m + 2,
 *     Dhat = I - c^-2 H_eo H_oe,  bhat = b_e / c + c^-2 H_eo b_o,
 * and reconstructs x_o = b_o / c + c^-1 H_oe x_e.
 *
 * Layouts (all complex numbers are complex128, interleaved (re, im)):
 *   gauge    U[mu][y][x]      mu = 0: link (x,y)->(x+1,y), mu = 1: (x,y)->(x,y+1)
 *                             (the U_mu^z of Sec. 2, Fig. 1)
 *   spinor   psi[y][x][s]     full lattice, 2 N^2 entries; batched: [nrhs][y][x][s]
 *   reduced  v[y][xh][s]      even sites only (x + y even), x = 2 xh + (y mod 2),
 *                             N^2 entries; batched: [nrhs][...]
 *   level l  v[site][d]       coarse level l >= 1: site = ay * ex + ax on an
 *                             ex x ey grid, d = 8 s + k (spin s, k < 8), 16 per site
 *   P_l      [agg][s][row][k] interpolation from level l+1 to level l per aggregate
 *                             and spin; row < 16 on level 0 (local even site
 *                             4*(y mod 4) + (xh mod 4)), row < 32 on coarser levels
 *                             (8 * local site + d mod 8, local site 2*(ay mod 2) + (ax mod 2))
 *   D_l      [site][o][i][j]  coarse operator (l >= 1) as 16x16 blocks coupling a
 *                             site to its neighbour at offset o in the order
 *                             (0,0) (+1,0) (-1,0) (0,+1) (0,-1) (+1,+1) (-1,-1)
 *
 * Pointers: unless stated otherwise every array argument is DEVICE memory
 * (for example torch.Tensor.data_ptr() of a CUDA/HIP tensor) that is valid on
 * the stream given in bamg_params.stream.  Host pointers are marked _host.
 * Ownership: the caller owns every array it passes; the library copies the
 * gauge field at setup and keeps no caller pointer after a call returns.  The
 * hierarchy is owned by the library until bamg_free.
 * Errors: every int-returning call returns a bamg_status.  Negative values are
 * failures (outputs unspecified); BAMG_NOT_CONVERGED leaves the best iterate.
 * bamg_last_error() returns a thread-local text for the last failure.
 * Threads and streams: one hierarchy must not be used from two threads at
 * once; different hierarchies may run concurrently on different streams.
 */
#ifndef BAMG_H
#define BAMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bamg_hierarchy bamg_hierarchy;

typedef enum {
  BAMG_OK = 0,
  BAMG_NOT_CONVERGED = 1,
  BAMG_PENDING = 2,        /* bamg_server_wait: the request is not finished yet */
  BAMG_EINVAL = -1,
  BAMG_ENOMEM = -2,
  BAMG_EDEVICE = -3,
  BAMG_ESINGULAR = -4,
  BAMG_ENOTIMPL = -5
} bamg_status;

/* Cycle of the preconditioner (Sec. 1 two-grid scheme applied recursively; Sec. 4):
 *   V: one visit of the coarser level per visit of a level;
 *   W: two visits (the solve cycle of Sec. 4; on two levels the same as V);
 *   K: every level l >= 1 that is not the coarsest is visited by two steps of
 *      flexible GCR on its coarse system from a zero start, each preconditioned
 *      by one (K-)cycle from that level: z1 = M r0, w1 = A z1, a1 = <w1, r0>/<w1, w1>,
 *      r1 = r0 - a1 w1, z2 = M r1, w2 = A z2 made orthogonal to w1 (z2 alike),
 *      x = a1 z1 + a2 z2 with a2 = <w2, r1>/<w2, w2>.  The paper names no
 *      Krylov-accelerated cycle; this is the recursive Krylov cycle of the
 *      multigrid literature with a fixed two steps (no norm test), so that a
 *      visit is a fixed launch sequence.  It makes the preconditioner depend on
 *      its input nonlinearly, which the flexible outer GMRES allows. */
typedef enum { BAMG_CYCLE_V = 0, BAMG_CYCLE_W = 1, BAMG_CYCLE_K = 2 } bamg_cycle;

typedef enum {
  BAMG_FP64 = 0,        /* everything in FP64 */
  BAMG_MIXED_FP16 = 1,  /* FP64 outer FGMRES + coarsest solve (see coarsest_fp32); FP32 cycle; coarse
                           operators stored FP16 */
  BAMG_MIXED_BF16 = 2,  /* as above with BF16 storage */
  BAMG_MIXED_FP32 = 3   /* as above with FP32 storage */
} bamg_precision;

/* Aggregates are fixed (Sec. 3.3 aggregates, reading: 4 x 4 blocks): level 1 is
 * built from 4 x 4 blocks of the half-x grid of even sites (16 sites, 32 dofs,
 * 16 coarse dofs), every further level from 2 x 2 blocks of the sites below;
 * there is no per-level shape parameter.  Levels are added while the
 * extents stay even and >= 4 (up to n_levels, or until max_coarse). */
typedef struct {
  int32_t N;            /* lattice extent, N % 8 == 0, N >= 16 */
  int32_t n_levels;     /* 0: automatic (coarsen until the level dimension <= max_coarse) */
  int32_t max_coarse;   /* dimension bound of the directly solved coarsest level (default 8192, at most 8192) */
  int32_t n_tv;         /* test vectors k (Sec. 4: k_r = 8); must be 8 */
  int32_t setup_sweeps; /* Kaczmarz sweeps on A_l v = 0 per level and setup pass (default 20) */
  int32_t setup_adapt;  /* adaptive passes after the first setup pass (default 1) */
  int32_t pre, post;    /* smoothing sweeps of the solve cycle (default 4, 4; Sec. 4) */
  int32_t cycle;        /* bamg_cycle (default V) */
  int32_t precision;    /* bamg_precision (default FP64) */
  int32_t restart;      /* FGMRES restart length (default 32; Sec. 4) */
  int32_t max_iter;     /* FGMRES iteration cap (default 1000) */
  uint64_t seed;        /* Philox4x32-10 key of the random initial test vectors */
  const double *init_tv_host; /* optional HOST [n_tv][N*N] complex reduced vectors; overrides seed */
  void *stream;         /* hipStream_t for all work, or NULL for the null stream */
  int32_t graphs;       /* 1: replay each FGMRES iteration (cycle, Dhat, Gram-Schmidt, norms) as a
                           captured hipGraph, one per (iteration index | batch size); 0 (default):
                           launch the kernels one by one.  Results are bitwise the same. */
  int32_t setup_mode;   /* 0 (default): relax-fit passes (setup_sweeps, setup_adapt);
                           1: bootstrap W setup cycles with the multigrid eigensolver (Sec. 3.4,
                              Sec. 4.1): W(boot_nu1) cycle, adaptive step (two solve cycles on the
                              eigenvector approximation of smallest |Ritz value|), W(boot_nu2) cycle;
                           2: the same with super-V cycles, boot_nu 2^l sweeps on level l (Sec. 4.2) */
  int32_t n_ev;         /* k_e eigenvector approximations of the bootstrap modes (1..8, default 8) */
  int32_t boot_nu1, boot_nu2; /* sweeps of the two bootstrap setup cycles (default 10, 5) */
  int32_t coarsest_fp32; /* mixed precisions only.  0 (default): the cycle's coarsest solve applies the
                           FP64 inverse (FP64 in and out).  1: it reads FP32 copies of that inverse
                           (rounded to nearest), FP32 in and out: half the bytes of the coarsest read,
                           relative rounding 2^-24 per entry */
  int32_t lookahead;    /* bamg_solve only (one right-hand side; the batched solves are not affected).
                           1 (default): while the estimated residual exceeds 1000 tol, FGMRES iteration
                           j + 1 (its cycle, Dhat, Gram-Schmidt) is queued on the stream before the host
                           has read iteration j's norms, so that the host's convergence test overlaps
                           the device's work; if the test stops the solve, the queued iteration ran for
                           nothing (never used).  0: off.  2: at every iteration (a check that the
                           results do not depend on it).  Results are bitwise the same in all three. */
} bamg_params;

typedef struct {
  int32_t iters;          /* FGMRES iterations (preconditioner applications) */
  int32_t restarts;       /* restarts performed */
  double relres_reduced;  /* ||bhat - Dhat x_e|| / ||bhat|| (true residual) */
  double relres_full;     /* ||b - D x|| / ||b|| of the unreduced system (eq. wilson), computed on the
                             device after the reconstruction (one application of D); 0 for a
                             request that failed before x was written */
  double rho_est;         /* relres_reduced^(1/iters), the mean residual reduction per FGMRES
                             iteration (the convergence rate of Sec. 4 is bamg_stationary's) */
  double t_solve_ms;      /* host wall time of the call */
} bamg_solve_info;

/* Fill p with the defaults listed above (N = 0: the caller must set it). */
int bamg_default_params(bamg_params *p);

/* Build the hierarchy for gauge field `gauge` (device, U[mu][y][x]) and mass m
 * (Sec. 3.4 bootstrap setup, reading: relax k random test vectors with Kaczmarz
 * on A_l v = 0, least-squares fit of P per aggregate and spin (Sec. 3.3),
 * Galerkin coarse operators P^H A_l P (Sec. 3.5), direct coarsest solve,
 * followed by `setup_adapt` adaptive passes of two cycles per test vector).
 * Returns BAMG_EINVAL for bad parameters, BAMG_ESINGULAR if the coarsest
 * operator is singular, BAMG_ENOMEM / BAMG_EDEVICE on allocation or HIP errors. */
int bamg_setup(const void *gauge, double m, const bamg_params *p, bamg_hierarchy **out);

/* Solve D x = b for one right-hand side (device b and x, full-lattice layout).
 * tol is the relative residual of the reduced system (Sec. 4: ||r|| / ||bhat||).
 * info may be NULL.  BAMG_EINVAL if b holds a non-finite value. */
int bamg_solve(bamg_hierarchy *h, const void *b, void *x, double tol, bamg_solve_info *info);

/* nrhs independent solves with one shared hierarchy: B and X are [nrhs][y][x][s].
 * infos (host, may be NULL) receives nrhs records.  Each right-hand side
 * converges on its own (lockstep FGMRES with per-RHS bases) and its result is
 * bitwise independent of nrhs and of the other right-hand sides; it equals the
 * result of bamg_solve up to rounding (bamg_solve uses single-RHS kernels). */
int bamg_solve_batch(bamg_hierarchy *h, const void *B, void *X, int32_t nrhs, double tol,
                     bamg_solve_info *infos);

/* y = Dhat x on nrhs reduced vectors (Sec. 3.2, eq. wilsonSchur). */
int bamg_apply_dhat(bamg_hierarchy *h, const void *x, void *y, int32_t nrhs);

/* bhat = b_e / c + c^-2 H_eo b_o for nrhs full-lattice b (Sec. 3.2, step 1). */
int bamg_eo_reduce(bamg_hierarchy *h, const void *b, void *bhat, int32_t nrhs);

/* x (full lattice) from x_e: even sites copied, x_o = b_o / c + c^-1 H_oe x_e
 * (Sec. 3.2, step 2). */
int bamg_eo_reconstruct(bamg_hierarchy *h, const void *b, const void *xe, void *x, int32_t nrhs);

/* Level operations on nrhs level-l vectors (test and benchmark hook):
 *   op 0 BAMG_OP_APPLY:    out = A_l in
 *   op 1 BAMG_OP_SWEEP:    out <- one multicolour Kaczmarz sweep on A_l out = in (in place on out)
 *   op 2 BAMG_OP_RESTRICT: out (level l+1) = P_l^H in
 *   op 3 BAMG_OP_PROLONG:  out (level l) += P_l in (level l+1)
 *   op 4 BAMG_OP_COARSEST: out = A_L^-1 in  (l must be the coarsest level).  For nrhs <= 2
 *         and a dimension that is a multiple of 64 the product reads only the 64 x 64
 *         blocks on and above the diagonal of the inverse, which is gamma5-Hermitian
 *         like the coarsest operator (Sec. 3.5), and takes the others as their
 *         mirrors (each stored block is the average of A_IJ and the mirror of A_JI);
 *         else the whole inverse
 *   op 5 BAMG_OP_CYCLE:    out = one multigrid cycle from level l on A_l out = in, zero start
 *   op 6 BAMG_OP_RESIDUAL: out = in - A_l out  (in: right-hand side; out: iterate, overwritten)
 * Mixed-precision hierarchies only (in and out stay complex128; the work is
 * done in FP32 with the coarse operator in the hierarchy's storage type):
 *   op 7 BAMG_OP_APPLY_MIXED, op 8 BAMG_OP_SWEEP_MIXED: as ops 0 and 1 (l not the coarsest)
 *   op 9 BAMG_OP_CYCLE_MIXED: out = the preconditioner of the solve applied to in (l = 0)
 *   op 10 BAMG_OP_APPLY_F32, op 11 BAMG_OP_SWEEP_F32: as ops 7 and 8, but in and out
 *         are complex64 (interleaved float) arrays used as they are, with no
 *         conversion launches: exactly the kernels of one FP32 apply or sweep
 *   op 12 BAMG_OP_COARSEST_F32: out = A_L^-1 in with complex64 in and out
 *         (l the coarsest level, coarsest_fp32 = 1), read from the FP32 copies of
 *         the inverse that the mixed cycle then uses: for nrhs <= 2 the packed
 *         blocks of op 4 in FP32 (block product, then the reduction of its partial
 *         products), else the split-K product with the whole FP32 copy on the
 *         matrix cores and its reduction
 *   op 13 BAMG_OP_SWEEP_COLOURS: as op 1, but as one launch per colour (Sec. 3.1
 *         in its plain form), whatever the size: the reference for the fused
 *         forms that op 1 runs where they apply (level 0: a sweep blocked in LDS,
 *         streaming or pipelined; coarse levels: two colours per launch), which
 *         give the same bits
 *   op 14 BAMG_OP_SWEEP_COLOURS_F32: op 13 for op 11 (complex64 in and out,
 *         mixed hierarchies; the colour passes on the vector units for any nrhs)
 * Ops 4 and 12 require in and out not to alias.
 * Level 0 is the fine reduced system (A_0 = Dhat). */
enum { BAMG_OP_APPLY = 0, BAMG_OP_SWEEP = 1, BAMG_OP_RESTRICT = 2, BAMG_OP_PROLONG = 3,
       BAMG_OP_COARSEST = 4, BAMG_OP_CYCLE = 5, BAMG_OP_RESIDUAL = 6,
       BAMG_OP_APPLY_MIXED = 7, BAMG_OP_SWEEP_MIXED = 8, BAMG_OP_CYCLE_MIXED = 9,
       BAMG_OP_APPLY_F32 = 10, BAMG_OP_SWEEP_F32 = 11, BAMG_OP_COARSEST_F32 = 12,
       BAMG_OP_SWEEP_COLOURS = 13, BAMG_OP_SWEEP_COLOURS_F32 = 14 };
int bamg_level_op(bamg_hierarchy *h, int32_t level, int32_t op, const void *in, void *out, int32_t nrhs);

/* Pieces of the bootstrap multigrid eigensolver (Sec. 3.4, Theorem 1 of Sec. 3.5;
 * test hook), FP64, on k level-l vectors X (device, [k][n_l]) and host lam_host[k]:
 *   op 0 BAMG_BOOT_RITZ:   lam_host[r] = <Z_l x_r, x_r> / <x_r, x_r>, Z_l = Gamma_5 D_l (eq. eqevZ)
 *   op 1 BAMG_BOOT_SWEEP:  x_r <- one Kaczmarz sweep on (D_l - lam_r Gamma_5) x_r = 0 (l not coarsest)
 *   op 2 BAMG_BOOT_EIGS:   X = the k (<= 8) eigenvectors of Z_L with the smallest |lambda|, lam_host
 *                          their eigenvalues (l = L-1, the coarsest level)
 *   op 3 BAMG_BOOT_FIT:    P_l = least squares fit to the k (<= 16) test vectors X (rank-8 fit per
 *                          aggregate and spin); level l+1 is rebuilt (Galerkin, smoother data or inverse)
 * Gamma_5 is +1 on spin 0 and -1 on spin 1. */
enum { BAMG_BOOT_RITZ = 0, BAMG_BOOT_SWEEP = 1, BAMG_BOOT_EIGS = 2, BAMG_BOOT_FIT = 3 };
int bamg_boot_op(bamg_hierarchy *h, int32_t level, int32_t op, void *X, double *lam_host, int32_t k);

/* After a bootstrap setup (setup_mode 1 or 2): the k_e Ritz values (lam_host) and
 * level-0 eigenvector approximations (ve_host, [k_e][N*N], may be NULL); returns k_e. */
int bamg_export_boot(const bamg_hierarchy *h, double *lam_host, void *ve_host);

/* Number of levels, or a negative status. */
int bamg_n_levels(const bamg_hierarchy *h);

/* info_host[0..4] = ex, ey, dofs per site, level dimension, colours of the smoother. */
int bamg_level_info(const bamg_hierarchy *h, int32_t level, int32_t *info_host);

/* Copy level l to host buffers (any may be NULL): P_host = P_l (l < L-1), Dl_host =
 * D_l in blocks (l >= 1; the coarsest level too), tv_host = the level-0 test vectors
 * [n_tv][N*N] after the last setup pass (l == 0 only). */
int bamg_export_level(const bamg_hierarchy *h, int32_t l, void *P_host, void *Dl_host, void *tv_host);

/* Replace parts of level l from host buffers (at least one non-NULL):
 *   Dl_host (l >= 1): the coarse operator D_l in blocks [site][7][16][16] (the
 *     export layout); its smoother data, or on the coarsest level its inverse,
 *     is rebuilt from it.  BAMG_ESINGULAR if a coarsest D_l is singular.
 *   P_host (l < L-1): P_l in aggregate blocks; level l+1 is then rebuilt by the
 *     Galerkin product P_l^H D_l P_l (Sec. 3.5) of the current D_l, with its
 *     smoother data or inverse.
 * D_l is replaced first, so both together give D_{l+1} = P^H D_l P from the new
 * pair.  Levels below l+1 keep their old P and D and are rebuilt by importing
 * them in order. */
int bamg_import_level(bamg_hierarchy *h, int32_t l, const void *P_host, const void *Dl_host);

/* Stand-alone iteration of the solver (Sec. 4: the convergence rate
 * rho = ||e^nu|| / ||e^{nu-1}|| of BAMG used on its own): x <- x + M(0 - Dhat x)
 * on the reduced system, M the hierarchy's preconditioner (one cycle in its
 * precision, zero initial guess), `iters` times from x (device, reduced
 * vector, overwritten by the last iterate).  With b = 0 the iterate is the
 * error.  norms_host[i] = ||x|| after i iterations (iters + 1 entries), so the
 * rate of iteration i is norms_host[i] / norms_host[i-1]. */
int bamg_stationary(bamg_hierarchy *h, void *x, int32_t iters, double *norms_host);

/* Residual norms of the unreduced system (Sec. 2, eq. wilson), independent of
 * any hierarchy: relres[r] = ||b_r - D x_r|| / ||b_r|| (||b_r - D x_r|| where
 * b_r = 0) for nrhs full-lattice pairs, D = (m + 2) I - H with the gauge field
 * U[mu][y][x].  gauge, B, X ([nrhs][y][x][s]) and relres (nrhs doubles) are
 * device arrays; the work is queued on `stream` (NULL: the null stream) and
 * relres is valid when it completes.  The partial sums (2 * min(256,
 * ceil(N^2 / 1024)) doubles per right-hand side) are allocated and freed on
 * the stream by the call.  BAMG_EINVAL for bad sizes, BAMG_ENOMEM if the
 * partial sums cannot be allocated. */
int bamg_full_residual(int32_t N, const void *gauge, double m, const void *B, const void *X, int32_t nrhs,
                       double *relres, void *stream);

/* bamg_full_residual for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and result, with the partial sums in a static device array
 * of 1 MiB per GPU (131072 doubles) that the library holds until the process
 * ends; the call allocates nothing.  It needs 2 * min(256, ceil(N^2 / 1024))
 * doubles per right-hand side (at most 256 right-hand sides for N >= 512) and
 * returns BAMG_EINVAL beyond that.  The array belongs to the current device,
 * which `stream` must be on.  Calls that overlap on one GPU share the array
 * and race: order them (one stream, or synchronise between them). */
int bamg_full_residual_noalloc(int32_t N, const void *gauge, double m, const void *B, const void *X,
                               int32_t nrhs, double *relres, void *stream);

/* Device bytes a hierarchy with parameters p holds after bamg_setup and a first
 * single-RHS solve: every level's data and work vectors (sized for the setup's
 * n_tv + n_ev test vectors), the FP32 copies of the mixed modes, the coarsest
 * inverse with its packed half and scratch, the bootstrap eigensolver's blocks and the FGMRES
 * workspace of one right-hand side.  0 for invalid parameters.  Batched solves
 * add workspace per right-hand side. */
size_t bamg_footprint_bytes(const bamg_params *p);

/* The tile plan of the level-0 Kaczmarz sweep blocked in LDS (Sec. 3.1; one
 * launch per 16-colour sweep, bitwise the colour-by-colour sweep), host only.
 * The even sites are addressed by u = (x + y)/2, v = (x - y)/2, the colour is
 * 4 (u mod 4) + (v mod 4); tiles of Tu x Tv sites start at u0 = 1 + a Tu,
 * v0 = 1 + b Tv (a < ntu = N / Tu, b < ntv = N / 2 / Tv).  A tile's work-group
 * reads the region [u0 + i0, u0 + i0 + Ru) x [v0 + j0, v0 + j0 + Rv) of x,
 * projects, for colour c = 0..15, the sites u0 + si0[c] + 4 p, v0 + sj0[c] + 4 q
 * (p < (first[c+1] - first[c]) / nj[c], q < nj[c]) in this order, and writes
 * its own tile.  The pipelined form (3) marches its tile's region down v
 * with a ring of W columns: colour c projects column sj0[c] + 4k at
 * macro-step c + k (k < nj[c]), all rows of a macro-step at once; region
 * column j0 + j is read at macro-step max(0, floor((j0 + j - A) / 4)) into
 * ring slot j mod W, whose previous column (j - W) is written out first if it
 * belongs to the tile; M macro-steps in all.
 *   form: 0 the library's choice for nrhs right-hand sides, 1 the
 *         LDS-resident form's tile, 2 the streaming form's tile, 3 the
 *         pipelined form's tile;
 *   fp32: nonzero for FP32 arithmetic (the mixed cycle), else FP64;
 *   plan_out (host, 77 int32): Tu, Tv, ntu, ntv, i0, j0, Ru, Rv, nupd,
 *         first[17], si0[16], sj0[16], nj[16] (nupd = first[16] projections),
 *         then A, M, W of form 3 (zeros for forms 1 and 2).
 * Returns the form of the plan written (1, 2 or 3), 0 if the colour passes
 * are used (form 0) or no tile applies (the lattice is too small or N/2 is
 * not a multiple of 8), BAMG_EINVAL for bad arguments. */
int bamg_fine_sweep_plan(int32_t N, int32_t nrhs, int32_t fp32, int32_t form, int32_t *plan_out);

/* k test vectors from the Philox4x32-10 generator (as used by setup):
 * out (device) [k][N*N] reduced vectors, entries (re, im) i.i.d. N(0, 1/2). */
int bamg_gaussian_tv(int32_t N, int32_t k, uint64_t seed, void *out, void *stream);

/* Release the hierarchy (NULL is ignored). */
void bamg_free(bamg_hierarchy *h);

/* ---- Serving: continuous batching over resident hierarchies ----------------
 * The paper's setting is many right-hand sides per gauge configuration (Sec. 1);
 * a server holds the hierarchies of several gauge fields (any lattice sizes,
 * masses and precisions) on the device and solves the right-hand sides of the
 * requests submitted for them as they arrive.
 *  - Memory admission: a field's hierarchy is built (bamg_setup) when a request
 *    for it is first scheduled and its footprint (hierarchy + slots_per_field
 *    solve slots, bamg_server_field_bytes) fits in hbm_budget beside the
 *    resident fields; idle resident fields are evicted, least recently used
 *    first, to make room.  A field larger than the whole budget fails its
 *    requests with BAMG_ENOMEM.
 *  - Continuous batching: every scheduling round moves queued right-hand sides
 *    into free slots of their field, then advances every occupied slot of every
 *    field by one FGMRES iteration (the fields' work overlaps on the device on
 *    one stream per field).  A request finishes when all its right-hand sides
 *    have.  Each right-hand side is solved exactly as by bamg_solve_batch: its
 *    result is bitwise the same alone or in any mix.
 *  - Pointers: B and X are DEVICE arrays [nrhs][y][x][s] (complex128) that must
 *    stay valid, with B unchanged and X untouched, until the request finishes;
 *    B must be complete (its producer synchronised) before bamg_server_submit.
 *  - Threads: with threaded = 1 a worker thread drives the device and
 *    bamg_server_wait blocks; with threaded = 0 the caller drives it with
 *    bamg_server_progress and bamg_server_wait only polls.  All calls may be made
 *    from any thread.  bamg_server_free stops the worker after its current round
 *    and drops unfinished requests. */
typedef struct bamg_server bamg_server;

typedef struct {
  size_t hbm_budget;        /* device bytes for hierarchies and slots (0: 80% of the free memory) */
  int32_t slots_per_field;  /* right-hand sides in flight per field (default 32, at most 4096) */
  int32_t threaded;         /* 1 (default): own worker thread; 0: driven by bamg_server_progress */
} bamg_server_params;

typedef struct {
  int64_t submitted, completed;     /* requests */
  int64_t rhs_completed;            /* right-hand sides of completed requests */
  double p50_ms, p99_ms, mean_ms, max_ms;  /* request latency, submit to completion (nearest rank) */
  double busy_s;                    /* first submit to last completion */
  double solves_per_s;              /* rhs_completed / busy_s */
  int32_t resident_fields, evictions, setups;
  size_t bytes_in_use, budget_bytes;
  int64_t rounds;                   /* scheduling rounds run */
} bamg_server_stats;

int bamg_server_default_params(bamg_server_params *sp);
int bamg_server_create(const bamg_server_params *sp, bamg_server **out);
/* Register a gauge field (device U[mu][y][x], copied to the host) with its mass
 * and hierarchy parameters (p->stream is ignored: each field gets a stream). */
int bamg_server_add_field(bamg_server *s, const void *gauge, double m, const bamg_params *p, int32_t *field_id);
/* Device bytes the field occupies while resident (admission footprint). */
int bamg_server_field_bytes(bamg_server *s, int32_t field_id, size_t *bytes);
/* Queue nrhs right-hand sides (1..4096) for a field; returns at once. */
int bamg_server_submit(bamg_server *s, int32_t field_id, const void *B, void *X, int32_t nrhs, double tol,
                       int64_t *request_id);
/* One scheduling round (threaded = 0 only); *pending (may be NULL) = unfinished requests. */
int bamg_server_progress(bamg_server *s, int32_t *pending);
/* Wait up to timeout_ms (< 0: forever) for a request.  Finished: its status
 * (BAMG_OK, BAMG_NOT_CONVERGED or a failure), infos_host[nrhs] filled (may be
 * NULL) and the request forgotten; else BAMG_PENDING. */
int bamg_server_wait(bamg_server *s, int64_t request_id, double timeout_ms, bamg_solve_info *infos_host);
int bamg_server_get_stats(bamg_server *s, bamg_server_stats *out);
/* Zero the statistics (counters and latencies); resident fields stay. */
int bamg_server_reset_stats(bamg_server *s);
void bamg_server_free(bamg_server *s);

/* Text of the last error on this thread ("" if none). */
const char *bamg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BAMG_H */
