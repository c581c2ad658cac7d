/*
 * dpg.h -- C ABI of libdpgmi: the per-cell local solve of the discontinuous
 * Petrov-Galerkin (DPG) method for the ultraweak time-harmonic Maxwell system
 * on hexahedra, on one AMD MI355X (gfx950) GPU.
 *
 * Method (Marquis, Maier, Blais, arXiv 2609.03155):
 *   For every cell K the library forms, from the cell's trilinear geometry,
 *   complex permittivity eps and permeability mu, frequency and trial degree p
 *   with test enrichment dp:
 *     G   -- Gram matrix of the enriched test space in the adjoint graph inner
 *            product (Sec. 2.2, test inner product, alpha > 0),
 *     B_f -- [B | Bhat]: the ultraweak bilinear form b_h and the skeleton trace
 *            pairing (Sec. 2.2), with entries as listed in Sec. 2.3,
 *     l   -- the linear form l_h (Sec. 2.2) with Robin data g,
 *   and returns (Sec. 2.3, elimination of the error representation function)
 *     K_e = B_f^H G^{-1} B_f,   l_e = B_f^H G^{-1} l,
 *     eta = ||Psi||_V = sqrt(r^H G^{-1} r),  r = B_f x - l  (Sec. 2.3).
 *   All forms are conjugate-linear in the first (test) argument.
 *
 * Conventions shared by every entry point
 *   - Units: non-dimensional as in App. A with the reference length given by
 *     the caller (the paper uses L = 1 m): x = x_dim / L,
 *     omega = L * 2*pi*freq / c0 with c0 = 299792458 m/s.
 *   - Complex numbers are interleaved (re, im) doubles.
 *   - Materials follow the paper's sign (time factor e^{-i omega t}): a lossy
 *     medium has Im(eps) > 0.
 *   - Reference cell [0,1]^3; cell vertex v(i,j,k) is entry 4k+2j+i of the
 *     cell's connectivity row; faces are numbered x-, x+, y-, y+, z-, z+.
 *   - Local unknown order (rows/columns of K_e, entries of l_e and x):
 *       E_x, E_y, E_z, H_x, H_y, H_z : (p+1)^3 discontinuous tensor-product
 *         Lagrange functions each, at the Gauss-Lobatto nodes, index
 *         i + (p+1)(j + (p+1)k) (x fastest);
 *       E-hat, H-hat : 12 (p+1)^2 tangential-trace functions each, from the
 *         first-kind Nedelec space of FEEC index r = p+1 mapped by the
 *         covariant Piola transform, interior functions dropped:
 *           12 edges x r functions  (edges 0-3 along x at (y,z) = (0,0),(1,0),
 *           (0,1),(1,1); 4-7 along y at (x,z); 8-11 along z at (x,y)); the
 *           function of degree i along the edge is
 *           sqrt(2i+1) P_i(2 xi_a - 1) * (vertex factors 1-xi or xi);
 *           then 6 faces x 2 r (r-1) functions: on face f with tangential
 *           axes t1 < t2, first the t1-component functions
 *           sqrt(2i+1)P_i(2xi_t1-1) * (1-xi_n or xi_n) * b_m(xi_t2), then the
 *           t2-component ones with t1 and t2 swapped; i = 0..r-1 fastest,
 *           m = 2..r; b_m(t) = (P_m(2t-1) - P_{m-2}(2t-1)) / sqrt(2(2m-1)).
 *     so k = 6 (p+1)^3 + 24 (p+1)^2 unknowns per cell.
 *   - Test space (internal; K_e, l_e and eta do not depend on its basis):
 *     first-kind Nedelec of FEEC index s = p+dp+1 for each of F and I,
 *     3 s (s+1)^2 functions per field.  Gauss-Legendre quadrature with
 *     p+dp+2 points per direction.
 *   - PEC faces are treated as interior faces locally (n x E = 0 is imposed
 *     on the global trace unknowns at assembly).  On Robin faces (port and
 *     impedance outlet) the H-hat pairing is absent, so H-hat functions that
 *     live only on Robin faces give zero rows and columns of K_e (Sec. 2.3).
 *   - Streams: every call that takes a stream enqueues its work on it and
 *     returns without synchronising; the caller owns all input and output
 *     buffers, the plan owns its scratch.  No C++ exception crosses the ABI.
 *   - Errors: argument errors are reported synchronously (DPG_ERR_ARG);
 *     HIP launch/allocation failures as DPG_ERR_HIP / DPG_ERR_ALLOC.
 *     Per-cell numerical failures never abort a batch; they are written to
 *     the device array info[] (0 = ok, -1 = degenerate cell geometry
 *     (det J <= 0 at a quadrature point or non-finite input), k > 0 = the
 *     Cholesky factorisation of the Jacobi-scaled G met a non-positive pivot
 *     at (1-based) column k of the padded test space).  Outputs of failed
 *     cells are unspecified.  dpg_sync waits for a stream and turns both
 *     kinds into a status: asynchronous HIP errors (DPG_ERR_HIP) and failed
 *     cells in info[] (DPG_ERR_CELL).
 */
#ifndef DPG_H
#define DPG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DPG_OK = 0,
  DPG_ERR_ARG = -1,          /* invalid argument (null pointer, bad degree, ...) */
  DPG_ERR_ALLOC = -2,        /* device or host allocation failed */
  DPG_ERR_HIP = -3,          /* a HIP runtime call or kernel launch failed */
  DPG_ERR_UNSUPPORTED = -4,  /* valid request the library does not support */
  DPG_ERR_CELL = -5          /* some cell failed (see info[]); returned by dpg_sync */
} dpg_status;

typedef enum {
  DPG_FP64 = 0,              /* every step in FP64 */
  DPG_SPLIT_FP32 = 1         /* split precision: formation, Cholesky and triangular solves in
                                FP64; K_e = W^H W and l_e = W^H y from a three-term bf16 split of
                                W (about 24 significant bits per operand, FP32 accumulation folded
                                into FP64 every 32 terms) on bf16 MFMA; eta by an FP64 reduction */
} dpg_precision;

enum {
  DPG_FACE_INTERIOR = 0,     /* interior skeleton face: trace pairing only */
  DPG_FACE_PEC = 1,          /* perfect conductor: local treatment as interior */
  DPG_FACE_PORT = 2,         /* Robin face, g from the TE_mn port mode */
  DPG_FACE_ROBIN0 = 3        /* Robin face with g = 0 (impedance outlet) */
};

/* TE_mn port mode of Sec. 4.1: a guide [0,a] x [0,b] (non-dimensional,
 * i.e. in units of L) along x3, filled with (eps, mu); the mode is the
 * paper's E_sol, H_sol with k_x1 = m pi/a, k_x2 = n pi/b,
 * k_x3 = sqrt(omega^2 eps mu - k_c^2) (principal branch).  On a DPG_FACE_PORT
 * face the Robin datum is g = n x H_sol + Z^{-1} n x (E_sol x n), with Z^{-1}
 * the face's admittance from dpg_problem.zinv. */
typedef struct {
  double a, b;
  int32_t m, n;
  double eps_re, eps_im;
  double mu_re, mu_im;
} dpg_port;

/* Problem description.  All arrays are DEVICE pointers (hipMalloc'ed or
 * torch CUDA tensors), read-only for the library. */
typedef struct {
  int64_t n_cells;
  int64_t n_vertices;
  const double* vertices;     /* [n_vertices][3], metres                       */
  const int64_t* cells;       /* [n_cells][8] vertex ids, v(i,j,k) at 4k+2j+i  */
  const double* eps;          /* [n_cells][2] complex relative permittivity    */
  const double* mu;           /* [n_cells][2] complex relative permeability    */
  const int8_t* face_kind;    /* [n_cells][6] DPG_FACE_* per face               */
  const double* zinv;         /* [n_cells][6][2] complex Robin admittance Z^-1 */
  double freq_hz;             /* excitation frequency                            */
  double length_m;            /* reference length L of App. A (paper: 1.0)      */
  double alpha;               /* L2 weight of the test norm (paper: 1.0), > 0   */
  dpg_port port;              /* mode used on DPG_FACE_PORT faces                */
} dpg_problem;

typedef struct dpg_plan_s* dpg_plan;
typedef struct dpg_graph_s* dpg_graph;
typedef struct dpg_trace_system_s* dpg_trace_system;

/* Local sizes of a (p, dp) cell (Sec. 2.3 spaces): n_test = 6 s (s+1)^2
 * (F and I), n_interior = 6 (p+1)^3 (E and H), n_trace = 24 (p+1)^2
 * (E-hat and H-hat).  Supported: 1 <= p <= 4, 1 <= dp <= 2.  Host only. */
dpg_status dpg_local_dims(int32_t p, int32_t dp, int32_t* n_test, int32_t* n_interior,
                          int32_t* n_trace);

/* Creates a plan for a batch of cells on HIP device `device`.
 * degree_host: HOST array [n_cells] of trial degrees p (1..4); dp: the test
 * enrichment (1..2) used for every cell.  The plan groups cells by degree
 * (the batching of the mixed-degree cells of Sec. 3's workloads, which the
 * per-cell solve of Sec. 2.3 leaves free), orders the groups by decreasing
 * algorithmic cost (the work queue), builds the reference tables of each
 * degree on the device and gives each group its own workspace: room for
 * enough cells that a factorisation step has about 16384 row tiles (at
 * least 64 cells, at most all of them), plus a share of the rest of
 * max_workspace_bytes
 * (0 = 40% of the device memory free at creation) proportional to the
 * group's cost and capped at what all its cells need (all scaled down if
 * the budget is short); a group with more cells than its workspace holds
 * is solved in chunks.  Each
 * group also gets a branch stream of default priority.  Synchronous. */
dpg_status dpg_plan_create(int32_t device, const int8_t* degree_host, int64_t n_cells, int32_t dp,
                           int64_t max_workspace_bytes, dpg_plan* plan);

dpg_status dpg_plan_destroy(dpg_plan plan);

/* Output offsets, in complex elements, written to HOST arrays of n_cells+1
 * entries: K_e of cell c occupies K[K_off[c] .. K_off[c+1]) (k_c x k_c,
 * column-major, full Hermitian), l_e and x of cell c occupy
 * [v_off[c] .. v_off[c+1]) (k_c entries). */
dpg_status dpg_plan_offsets(dpg_plan plan, int64_t* K_off, int64_t* v_off);

/* Number of padded test rows, RHS rows and cells per chunk used for degree p
 * (diagnostics and tests).  Host only. */
dpg_status dpg_plan_layout(dpg_plan plan, int32_t p, int64_t* n_test_padded, int64_t* n_rhs_padded,
                           int64_t* chunk_cells);

/* The local solve.  Device pointers:
 *   x    [v_off[n]][2]  trial + trace coefficients per cell for eta, or NULL
 *                       (then eta is written as 0),
 *   K    [K_off[n]][2]  K_e per cell (output),
 *   l    [v_off[n]][2]  l_e per cell (output),
 *   eta  [n]            residual indicator per cell (output),
 *   info [n]            per-cell status (output, see above).
 * precision: DPG_FP64 or DPG_SPLIT_FP32 (DPG_ERR_ARG otherwise).
 * stream is a hipStream_t (NULL = the default stream). */
dpg_status dpg_local_solve(dpg_plan plan, const dpg_problem* prob, const double* x, double* K,
                           double* l, double* eta, int32_t* info, int32_t precision, void* stream);

/* The local solve of the cells first .. first+count-1 only, for streaming
 * through batches whose outputs do not fit in memory at once.  Output and
 * coefficient pointers refer to the range: K_e of cell c starts at
 * K + 2*(K_off[c] - K_off[first]) doubles, l_e and x of cell c at
 * l + 2*(v_off[c] - v_off[first]), eta and info of cell c at index c - first.
 * Same stream, precision and error behaviour as dpg_local_solve. */
dpg_status dpg_local_solve_range(dpg_plan plan, const dpg_problem* prob, int64_t first, int64_t count,
                                 const double* x, double* K, double* l, double* eta, int32_t* info,
                                 int32_t precision, void* stream);

/* Degree groups of one solve run on parallel branches (enable = 1, the
 * default): each group's launches go to its own stream, forked from and
 * joined back into the caller's stream with events; with enable = 0 the
 * groups run one after the other on the caller's stream.  Results are the
 * same bit for bit either way.  Host only; affects later solves and graphs. */
dpg_status dpg_plan_set_concurrency(dpg_plan plan, int32_t enable);

/* Autotuner of the batching and tile shapes: after one warm-up solve, for
 * each degree group (queue order) it times whole solves of all n_cells cells
 * with 1, 1/2 and 1/4 of the group's chunk per launch sequence and keeps the
 * fastest; then, for each group, the tile shape of the sum-factorised
 * formation (8 or 4 column tiles of 16 per chunk, see dpg_plan_tiles) and
 * keeps the faster; then times the concurrent schedule against the
 * sequential one and keeps the faster.  Results do not depend on any of
 * these choices (bit for bit).
 * Arguments as dpg_local_solve (all cells); the outputs hold a complete
 * solve with the chosen settings on return.  *best_ms (may be NULL)
 * receives the time of that last solve.  Synchronises `stream`. */
dpg_status dpg_plan_autotune(dpg_plan plan, const dpg_problem* prob, const double* x, double* K, double* l,
                             double* eta, int32_t* info, int32_t precision, void* stream, double* best_ms);

/* Current batching of degree p: cells per launch sequence and whether the
 * concurrent schedule is on.  Host only. */
dpg_status dpg_plan_tuning(dpg_plan plan, int32_t p, int64_t* run_chunk, int32_t* concurrent);

/* Tile shape of degree p's sum-factorised formation (the contractions of the
 * test-norm and trial-to-test forms, Sec. 2.2): the number of 16-column MFMA
 * tiles per chunk of the last contraction, 8 (the default) or 4 (less LDS
 * per workgroup, more workgroups per CU); wider blocks are never split.
 * dpg_plan_set_tiles sets it (DPG_ERR_ARG for other values or a degree the
 * plan does not hold); dpg_plan_autotune picks it.  Results are the same bit
 * for bit with either.  Host only; affects later solves and graphs. */
dpg_status dpg_plan_tiles(dpg_plan plan, int32_t p, int32_t* form_col_tiles);
dpg_status dpg_plan_set_tiles(dpg_plan plan, int32_t p, int32_t form_col_tiles);

/* Captures dpg_local_solve_range(plan, prob, first, count, x, K, l, eta,
 * info, precision) into a HIP graph (degree groups as parallel branches when
 * concurrency is on) for replay with dpg_graph_launch.  The graph keeps the
 * pointers it was captured with and the plan's workspace: the plan and the
 * buffers must outlive it, and replays, solves and other graphs of the same
 * plan must not overlap in time (they share the workspace).  Profiling is
 * not recorded inside graphs.  Synchronous (capture happens on a private
 * stream; nothing runs until a launch).  count = 0 gives an empty graph. */
dpg_status dpg_graph_create(dpg_plan plan, const dpg_problem* prob, int64_t first, int64_t count,
                            const double* x, double* K, double* l, double* eta, int32_t* info,
                            int32_t precision, dpg_graph* graph);

/* Enqueues one replay of the graph on `stream` (a hipStream_t, NULL = the
 * default stream). */
dpg_status dpg_graph_launch(dpg_graph graph, void* stream);

dpg_status dpg_graph_destroy(dpg_graph graph);

/* Debug/parity entry: the unscaled local matrices of `count` consecutive
 * cells first, first+1, ... which must all have the plan's degree p.
 * Device outputs, complex, column-major per cell:
 *   G [count][n_test][n_test], Bf [count][k][n_test] (column a of B_f is
 *   contiguous: Bf[c][a][i] = B_f(i, a)), lvec [count][n_test].
 * Row order of the test space: F functions (3 s (s+1)^2, component-major,
 * then x-, y-, z-degree with x fastest, orthonormal shifted Legendre factors),
 * then I functions in the same order.  info [count]: geometry status of cell
 * first + c at index c.  Synchronises `stream`. */
dpg_status dpg_form_local(dpg_plan plan, const dpg_problem* prob, int64_t first, int64_t count,
                          double* G, double* Bf, double* lvec, int32_t* info, void* stream);

/* Debug/parity entry: the Jacobi-scaled system of `count` consecutive cells
 * first, ... (all of the plan's degree p) exactly as the factorisation of
 * dpg_local_solve reads it, so that an independent solve of these FP64
 * numbers measures the factorisation's own error (Sec. 2.3: K_e, l_e and
 * eta are invariant under the scaling):
 *   Gs = D G D (full Hermitian, built from the lower triangle the
 *        factorisation reads), Bs = D B_f, ls = D l, rs = D (B_f x - l)
 *        (zero when x is NULL), d = diag(G)^{-1/2} (real).
 * Layouts as dpg_form_local (Gs [count][n_test][n_test], Bs [count][k][n_test],
 * ls and rs [count][n_test], complex; d [count][n_test] doubles); x, if not
 * NULL, holds the coefficients of the range (cell first + c at
 * x + 2*(v_off[first + c] - v_off[first])).  All device pointers.
 * Synchronises `stream`.  DPG_ERR_ARG as dpg_form_local, or for NULL rs or d. */
dpg_status dpg_form_augmented(dpg_plan plan, const dpg_problem* prob, int64_t first, int64_t count,
                              const double* x, double* Gs, double* Bs, double* ls, double* rs, double* d,
                              int32_t* info, void* stream);

/* ---------------------------------------------------------------------
 * Condensed trace system (Sec. 2.3: static condensation of the interior
 * unknowns; the global system in the trace unknowns that the paper solves
 * by CG).  Cell matrices are ordered as K_e: interior [E, H] (n_u = 6 (p+1)^3)
 * then trace [Ehat, Hhat] (n_t = 24 (p+1)^2), so
 *   K_e = [[M1, M2], [M2^H, M3]],  l_e = [l_u ; l_t].
 * --------------------------------------------------------------------- */

/* Offsets, in complex elements, of the condensed cell outputs, written to
 * HOST arrays of n_cells+1 entries: A_K of cell c occupies
 * A[A_off[c] .. A_off[c+1]) (n_t x n_t, column-major, full Hermitian), b_K
 * occupies b[b_off[c] .. b_off[c+1]) (n_t entries). */
dpg_status dpg_plan_trace_offsets(dpg_plan plan, int64_t* A_off, int64_t* b_off);

/* Condensation of every cell (Sec. 2.3):
 *   A_K = M3 - M2^H M1^{-1} M2,   b_K = l_t - M2^H M1^{-1} l_u,
 * from the K_e, l_e a dpg_local_solve of the same plan wrote (device, its
 * layout).  On the GPU: a Jacobi-scaled blocked Cholesky of M1 with the rows
 * (D M2)^H, (D l_u)^H appended (the local solve's factorisation kernels),
 * a HERK of those rows, and the subtraction.  A, b: device outputs at the
 * dpg_plan_trace_offsets offsets; info [n_cells]: 0, or the failing pivot
 * column + 1 of M1.  Uses the plan's workspace (do not overlap with a solve
 * of the same plan).  Stream-ordered. */
dpg_status dpg_condense(dpg_plan plan, const double* K, const double* l, double* A, double* b, int32_t* info,
                        void* stream);

/* Numbering of the global trace unknowns and the CSR structure of
 *   A = sum_K P_K^T A_K P_K,  b = sum_K P_K^T b_K
 * for the plan's cells.  cells_host [n][8] (vertex ids, v(i,j,k) at 4k+2j+i)
 * and face_kind_host [n][6] are HOST arrays.  Rules:
 *   - local trace functions of a cell (Ehat then Hhat, 12 r^2 each) live on
 *     its 12 edges (r each; edges along x at (y,z) = (0,0),(1,0),(0,1),(1,1),
 *     then along y, then z) or 6 faces (2 r (r-1) each; faces x-,x+,y-,y+,
 *     z-,z+; first the functions whose component is the lower tangential
 *     axis, then the other; bubble degree 2..r; along-degree fastest);
 *   - edges are identified by their (start, end) vertices along the local
 *     component axis and faces by their vertex sets; all cells must agree on
 *     edge directions and face axes (structured meshes do), else DPG_ERR_ARG;
 *   - minimum rule for mixed degrees: an edge or face keeps the functions of
 *     the smallest r among its cells, higher ones are constrained to zero;
 *   - removed (homogeneous Dirichlet) unknowns: Ehat on every edge or face
 *     inside a PEC face; Hhat face functions of Robin faces and Hhat edge
 *     functions whose cell faces are all Robin (they have zero rows, the
 *     pairing excludes Hhat there, Sec. 2.2);
 *   - kept unknowns are numbered in order of first appearance (cells in
 *     order, local functions in order); CSR columns ascend within a row.
 * Builds on the host (synchronous) and uploads the structure and the gather
 * lists of the assembly to the plan's device. */
dpg_status dpg_trace_system_create(dpg_plan plan, const int64_t* cells_host, const int8_t* face_kind_host,
                                   dpg_trace_system* sys);
/* The same numbering without a device: HOST arrays; glob receives
 * sum_c 24 (p_c+1)^2 ids (cell by cell, Ehat then Hhat), *n_dofs the number
 * of kept unknowns.  DPG_ERR_ARG for degrees outside 1..4 or inconsistent
 * orientations. */
dpg_status dpg_trace_numbering(const int64_t* cells_host, const int8_t* face_kind_host, const int8_t* degree_host,
                               int64_t n_cells, int64_t* glob, int64_t* n_dofs);
dpg_status dpg_trace_system_destroy(dpg_trace_system sys);
/* Number of unknowns and of stored nonzeros (host). */
dpg_status dpg_trace_system_info(dpg_trace_system sys, int64_t* n_dofs, int64_t* nnz);
/* HOST copy of the global id of every local trace function, laid out like b
 * (b_off), -1 where removed or constrained. */
dpg_status dpg_trace_system_numbering(dpg_trace_system sys, int64_t* glob);
/* DEVICE pointers to the CSR structure (row_ptr [n_dofs+1], col [nnz]),
 * owned by the system. */
dpg_status dpg_trace_system_csr(dpg_trace_system sys, const int64_t** row_ptr, const int32_t** col);

/* Assembly by gathering: vals [nnz] (complex) and rhs [n_dofs] (complex)
 * from the condensed cell outputs A, b (device); each entry is the sum of its
 * cell contributions in a fixed order (deterministic).  Stream-ordered. */
dpg_status dpg_assemble(dpg_trace_system sys, const double* A, const double* b, double* vals, double* rhs,
                        void* stream);

/* y = A x for a complex CSR matrix (the CG matvec); all device pointers,
 * x and y complex [n_rows].  Stream-ordered. */
dpg_status dpg_csr_matvec(int64_t n_rows, const int64_t* row_ptr, const int32_t* col, const double* vals,
                          const double* x, double* y, void* stream);

/* ---------------------------------------------------------------------
 * Global solve (Sec. 2.3 and Algorithm 1: the condensed trace system is
 * Hermitian positive definite and solved by CG without a preconditioner;
 * the interior unknowns and the residual are then recovered cell by cell).
 * --------------------------------------------------------------------- */

/* Conjugate gradients for the complex Hermitian positive definite CSR system
 * A x = b (n_rows unknowns; row_ptr [n_rows+1], col [nnz], vals [nnz]
 * complex, b and x [n_rows] complex; all device pointers), without a
 * preconditioner:
 *   q = A p, alpha = r^H r / p^H q, x += alpha p, r -= alpha q,
 *   beta = r_new^H r_new / r^H r, p = r + beta p,
 * from the start x (in: initial guess, out: last iterate) until the
 * recursively updated residual satisfies ||r||_2 <= tol ||b||_2, or
 * max_iter iterations.  *iters receives the iterations done, *relres the
 * final ||r||_2 / ||b||_2 (0 for b = 0, where x is left unchanged).  No
 * iteration runs when the start already satisfies the test.  The scalars
 * stay on the device and every reduction has a fixed order (bitwise
 * reproducible); the host reads the convergence flag once per 16 iterations
 * while the next 16 are queued.  A must be Hermitian positive definite and
 * every col entry in [0, n_rows) (not checked on the device).  For an
 * arbitrary CSR system: allocates and frees 3 n_rows complex vectors,
 * O(n_rows / 256) partial sums and pinned host slots on every call (the
 * assembled trace system's CG, dpg_trace_system_cg, keeps them in the
 * system instead); returns after synchronising `stream`.  DPG_ERR_ARG for
 * null pointers, n_rows < 0, max_iter < 0 or tol < 0 (or NaN). */
dpg_status dpg_cg_solve(int64_t n_rows, const int64_t* row_ptr, const int32_t* col, const double* vals,
                        const double* b, double* x, double tol, int64_t max_iter, int64_t* iters,
                        double* relres, void* stream);

/* The same CG (Sec. 2.3: the condensed trace system solved without a
 * preconditioner) on the trace system's own CSR structure: vals [nnz] and
 * b [n_dofs] as dpg_assemble writes them, x [n_dofs] (start in, solution
 * out), all device, complex.  Its vectors, partial sums, scalars, pinned host
 * slots and events were allocated with the system (dpg_trace_system_create),
 * so a call allocates nothing; calls on one system must not overlap in time.
 * Returns after synchronising `stream`.  Errors as dpg_cg_solve. */
dpg_status dpg_trace_system_cg(dpg_trace_system sys, const double* vals, const double* b, double* x, double tol,
                               int64_t max_iter, int64_t* iters, double* relres, void* stream);

/* The cells' local trace coefficients t_K = P_K t from the global trace
 * vector t (device, complex [n_dofs]): t_local (device, complex) is laid out
 * like the condensed right-hand sides (dpg_plan_trace_offsets' b_off), zero
 * where a local function is removed or constrained.  Stream-ordered. */
dpg_status dpg_trace_system_scatter(dpg_trace_system sys, const double* t, double* t_local, void* stream);

/* Interior unknowns of every cell from its traces (Sec. 2.3):
 *   u_K = M1^{-1} (l_u - M2 t_K),  K_e = [[M1, M2], [M2^H, M3]], l_e = [l_u ; l_t],
 * with K, l the outputs of a dpg_local_solve of the same plan (device, its
 * layout) and t_local the traces in the b_off layout (dpg_trace_system_scatter).
 * Writes x (device, complex, the v_off layout of the local solve's x and l:
 * k = n_u + n_t per cell) = [u_K ; t_K], the whole coefficient vector of the
 * cell, which a dpg_local_solve with this x turns into the residual
 * indicator eta of the global solution.  On the GPU: a Jacobi-scaled blocked
 * Cholesky of M1 with the row (D (l_u - M2 t_K))^H appended (the local
 * solve's factorisation kernels), then a backward substitution.  info
 * [n_cells]: 0, or the failing pivot column + 1 of M1.  Uses the plan's
 * workspace (do not overlap with another call on the same plan).
 * Stream-ordered. */
dpg_status dpg_reconstruct(dpg_plan plan, const double* K, const double* l, const double* t_local, double* x,
                           int32_t* info, void* stream);

/* Electromagnetic power dissipated in every cell (Sec. 3.2: the heat source
 * Q_em = sigma |E|^2/2 + omega eps0 eps_im |E|^2/2 + omega mu0 mu_im |H|^2/2,
 * the time average of minus the divergence of the Poynting vector), from the
 * cells' coefficient vectors x (device, complex, the v_off layout of a
 * dpg_local_solve's x, e.g. dpg_reconstruct's output; only the interior
 * part [E_x, E_y, E_z, H_x, H_y, H_z] is read).  In the non-dimensional
 * variables (lengths in units of L, E in units of E0, H of E0/Z0,
 * omega = 2 pi f L / c0, conductivity inside eps_im) the density is
 * q = omega (eps_im |E|^2 + mu_im |H|^2) / 2 and Q_em = q E0^2 / (Z0 L).
 * power [n_cells][3] (device): the cell integrals of q, |E|^2 and |H|^2, by
 * the volume Gauss rule of the local solve (exact for them on trilinear
 * cells).  Stream-ordered. */
dpg_status dpg_power_dissipation(dpg_plan plan, const dpg_problem* prob, const double* x, double* power,
                                 void* stream);

/* Dörfler marking for adaptive refinement (Sec. 4.2, the Fichera case, and
 * its refinement table: fractions 0.30 and 0.05).  values [n] (device,
 * finite, >= 0): one indicator per cell, e.g. the residual norm eta of a
 * dpg_local_solve (or its square, for marking by eta^2).  Cells are ranked by
 * decreasing value, equal values by increasing cell index; with T the sum of
 * all values and S the sum of those ranked before a cell,
 *   flags[i] = +1 (refine)  if S < refine_fraction T,
 *            = -1 (coarsen) if not refined and T - S <= coarsen_fraction T,
 *            =  0 otherwise
 * (flags [n], device, int8): the shortest prefix of the ranking that carries
 * refine_fraction of the total is refined, the longest run of the smallest
 * values within coarsen_fraction of it is coarsened.  The sums run in a fixed
 * order, so equal inputs give equal flags.  Temporaries (about 40 n bytes
 * and the radix sort's own): `workspace` (device, 256-byte aligned, at least
 * dpg_dorfler_mark_workspace_size(n) bytes, owned by the caller, e.g. kept
 * with the plan whose eta it marks), and then the call allocates nothing and
 * is stream-ordered; or, with workspace null, an allocation per call, after
 * which the call synchronises `stream`.  DPG_ERR_ARG for n < 0 or
 * n > 2^31 - 1, null pointers, fractions outside [0, 1], or a workspace
 * that is too small or misaligned (nothing is enqueued then). */
dpg_status dpg_dorfler_mark_workspace_size(int64_t n, size_t* bytes);
dpg_status dpg_dorfler_mark(int64_t n, const double* values, double refine_fraction, double coarsen_fraction,
                            int8_t* flags, void* workspace, size_t workspace_bytes, void* stream);

/* Dörfler marking without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same flags as dpg_dorfler_mark
 * (bit for bit) from the same values and fractions, but its temporaries (sort keys and
 * cell ids, chunk sums, the sort's own temporaries) live in a static device
 * array of 64 MiB on every GPU the library runs on, held until the process
 * ends; its device address is looked up once per device on the first call.
 * n <= 1048576 (2^20) cells; larger n, or temporaries beyond the array,
 * return DPG_ERR_UNSUPPORTED before anything is enqueued.  Stream-ordered:
 * returns without synchronising.  Every call on one GPU uses that GPU's one
 * array, so calls that overlap in time on the same GPU race (order them on
 * one stream).  Other errors as dpg_dorfler_mark. */
dpg_status dpg_dorfler_mark_noalloc(int64_t n, const double* values, double refine_fraction,
                                    double coarsen_fraction, int8_t* flags, void* stream);

/* Kernel classes timed by the plan's optional profiler. */
enum {
  DPG_K_SCALE = 0,      /* geometry check and Jacobi scaling            */
  DPG_K_FORM_SM = 1,    /* G_FF, G_II (volume and Robin mass terms)      */
  DPG_K_FORM_IF = 2,    /* G_IF from the geometry-free matrices          */
  DPG_K_FORM_PAD = 3,   /* padding of the test space                     */
  DPG_K_FORM_B = 4,     /* rows of B_f^H                                 */
  DPG_K_FORM_LOAD = 5,  /* port load vector                              */
  DPG_K_RESID = 6,      /* r = B_f x - l                                 */
  DPG_K_CHOL_DIAG = 7,  /* diagonal blocks of the blocked Cholesky       */
  DPG_K_CHOL_PANEL = 8, /* panels of L and of W^H (Cholesky + TRSM)      */
  DPG_K_HERK = 9,       /* K_aug = W^H W -> K_e, l_e, eta                */
  DPG_K_COUNT = 10
};

/* Enables (1) or disables (0) per-kernel timing: while enabled, every kernel
 * launch of dpg_local_solve is bracketed by HIP events recorded on the
 * stream it runs on (a group's branch stream under the concurrent schedule,
 * where concurrent kernels share the device).  Host only; takes effect for
 * later solves. */
dpg_status dpg_plan_set_profiling(dpg_plan plan, int32_t enable);

/* Waits for the recorded events and returns, per kernel class, the summed
 * device time in milliseconds (ms[DPG_K_COUNT]) and the number of launches
 * (launches[DPG_K_COUNT]) since the previous call; then resets.  Host only,
 * synchronises with the recorded events. */
dpg_status dpg_plan_profile(dpg_plan plan, double* ms, int64_t* launches);

/* Synchronises `stream` (a hipStream_t, NULL = the default stream) and
 * reports what the work enqueued on it left: DPG_ERR_HIP if the stream or a
 * kernel on it failed (an asynchronous HIP error; text in dpg_last_error),
 * else DPG_ERR_CELL if any of info[0..n) (a device array written by a solve,
 * range solve, condensation or reconstruction) is nonzero, else DPG_OK.
 * *n_failed (may be NULL) receives the number of nonzero entries and
 * *first_failed (may be NULL) the index of the first one (-1 if none).
 * info may be NULL when n = 0.  DPG_ERR_ARG for n < 0 or a NULL info with
 * n > 0.  Host only; reads info[] back through host memory (4 n bytes). */
dpg_status dpg_sync(void* stream, const int32_t* info, int64_t n, int64_t* n_failed, int64_t* first_failed);

const char* dpg_status_string(dpg_status s);

/* Text of the last HIP failure seen by this thread inside the library (the
 * failing call and HIP's error string), for diagnostics.  Host only. */
const char* dpg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DPG_H */
