/*
 * tnfem.h -- C ABI of the MI355X QTT finite-element elasticity solver.
 *
 * The library solves the Galerkin system A u = M f0 of isotropic linear
 * elasticity discretised by Q1 (bilinear / trilinear) elements on a box with
 * 2^d nodes per axis (Sec. 3 and Sec. 5 of Ali et al., "Quantum-Inspired Solver
 * for Simulating Material Deformations", arXiv 2501.12151), entirely in
 * quantics tensor-train (QTT) format, with the alternating minimal-energy
 * (AMEn) sweep that the paper's Alg. 2 applies.  Every step of the sweep runs in
 * the library's own HIP kernels for gfx950; the host only sequences them.
 *
 * Conventions
 * -----------
 * - All calls return an int status: TNFEM_OK (0) or a negative TNFEM_E* code;
 *   tnfem_last_error() then returns a message for the calling thread.
 * - Every *_create has a matching *_destroy.  Input arrays are caller owned and
 *   copied; output TTs are library owned until destroyed.
 * - Floating point is IEEE double unless stated otherwise.
 * - TT layout (the same for the solution u and the load b): K = d + 1 cores.
 *   Cores 0 .. d-1 are level cores with mode n = 2^D, most significant level
 *   first (the binary index formula of Sec. 4), mode index
 *   m = (ix_bit * 2 + iy_bit) [* 2 + iz_bit]; core d is the displacement
 *   component core with mode D.  (Sec. 5.2 lists the component index first;
 *   the library places it last, where the exact operator has lower TT rank:
 *   25 instead of 51 in 2D, 125 instead of 342 in 3D.)  Core k is stored
 *   row-major as [r_k][n_k][r_{k+1}], r_0 = r_K = 1.
 *   Node (ix, iy[, iz]) sits at x = ix * extent[0] / (2^d - 1), etc.
 * - Pointers documented as "device" are HIP device pointers on the context's
 *   device (for instance torch tensor data pointers); "host" pointers are
 *   ordinary memory.  A "stream" argument is a hipStream_t passed as void*;
 *   NULL means the context's stream.
 */
#ifndef TNFEM_H
#define TNFEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  TNFEM_OK = 0,
  TNFEM_EINVAL = -1,   /* invalid argument or descriptor */
  TNFEM_ENOMEM = -2,   /* host or device allocation failed */
  TNFEM_EBUDGET = -3,  /* request does not fit the device-memory budget */
  TNFEM_ENOTCONV = -4, /* sweep limit reached before the tolerance (result still returned) */
  TNFEM_EDEVICE = -5,  /* a HIP call failed, or no device */
  TNFEM_ENAN = -6,     /* a non-finite value appeared in the sweep */
  TNFEM_EBUSY = -7     /* result not ready yet (serving queue) */
};

typedef struct tnfem_ctx tnfem_ctx;
typedef struct tnfem_problem tnfem_problem;
typedef struct tnfem_tt tnfem_tt;

/* Face numbering: face = 2 * axis + side, side 0 at x_axis = 0, side 1 at x_axis = extent. */
#define TNFEM_FACE(axis, side) (2 * (axis) + (side))

/*
 * Problem description (Alg. 1 inputs: grid exponent d, Young's modulus E,
 * Poisson's ratio nu, domain, Dirichlet or Neumann data per side; Alg. 2 adds
 * the load).  Material law of Sec. 2: lambda = E nu / ((1+nu)(1-2nu)),
 * mu = E / (2(1+nu)); plane_stress (2D only) uses lambda = E nu / (1 - nu^2).
 * Clamped faces fix every displacement component (u = 0) by symmetric
 * elimination; other faces are traction free unless a traction is given.
 * Loads: body force f (constant vector, enters as b = M f0 with f0 its nodal
 * values, Sec. 5.3), uniform tractions t on faces (b += integral of t . v),
 * and the manufactured force of u*_i = c_i prod_a sin(pi x_a) on the unit box.
 * layer_E, if non-NULL, gives Young's modulus per element layer along
 * layer_axis (2^d - 1 values), i.e. a piecewise constant E(x) at fixed nu;
 * it replaces E in the element integrals (E still sets the diagonal given to
 * clamped dofs).  Only 2^d - 1 == n_layer_E is accepted.
 */
typedef struct {
  int dim;              /* D = 2 or 3 */
  int level;            /* d >= 2: 2^d nodes per axis, boundary nodes included */
  double extent[3];     /* box edge lengths (> 0) */
  double E, nu;         /* Young's modulus (> 0), Poisson's ratio in (-1, 0.5) */
  int plane_stress;     /* 2D only: 0 = plane strain, 1 = plane stress */
  uint32_t clamp_mask;  /* bit TNFEM_FACE(axis, side) set = clamped face */
  int n_tractions;      /* 0..6 */
  int traction_face[6];
  double traction[6][3];
  int has_body_force;
  double body_force[3];
  int has_manufactured;
  double manufactured_c[3];
  int layer_axis;
  int n_layer_E;
  const double* layer_E; /* host, n_layer_E values, copied */
  /* Optional nodal load f0 of Alg. 2 (Sec. 5.3): the body force at every node as a TT in
   * the layout of u (d level cores of mode 2^D, then the component core of mode D).
   * The load gains P M f0, M the consistent (vector) mass matrix and P the mask of the
   * dofs not clamped; the product is formed in TT format on the host (each axis' 1D
   * mass matrix as an exact rank <= 2 QTT operator per term) and rounded at 1e-14.
   * f0_ranks: d + 2 values, the first and last 1 (host, copied); f0_cores: all cores
   * concatenated, core k row-major [r_k][n_k][r_{k+1}] (host, copied).  f0_cores NULL:
   * no nodal load.  Invalid ranks fail with TNFEM_EINVAL. */
  const int* f0_ranks;
  const double* f0_cores;
  /* Optional anisotropic material (the non-isotropic materials of Sec. 7): the constant
   * stiffness in Voigt notation, sigma_V = C eps_V with engineering shear strains, order
   * (xx, yy, xy) in 2D (the leading 3 x 3 block is read) and (xx, yy, zz, yz, xz, xy) in
   * 3D.  It replaces the isotropic law built from E and nu in the element integrals
   * (layer_E / E still scales it per element layer); it must be symmetric positive
   * definite, and plane_stress must be 0 (a 2D C already states the plane assumption).
   * The clamped dofs get the diagonal max_i C_ii h^(D-2) (normal components i). */
  int has_stiffness;
  double stiffness[6][6];
  /* Optional quadrilateral domain (2D, Sec. 5: "any quadrilateral"): corners P00, P10, P01,
   * P11 (x, y), the images of the unit-square corners (s, t) = (0,0), (1,0), (0,1), (1,1)
   * under the bilinear map; node (i, j) sits at x(i / (2^d - 1), j / (2^d - 1)) and extent
   * is ignored.  Alg. 1 in full: element Jacobians and determinants at the element centres,
   * the coefficient fields over the element grid compressed to QTT, placed at node pairs by
   * corner-pair shift automata; clamps and tractions name the four sides as faces
   * (TNFEM_FACE(0, 0) is the side P00-P01, (0, 1) P10-P11, (1, 0) P00-P10, (1, 1) P01-P11;
   * a traction is per unit length of the side).  The corners must make every element's
   * det J positive (convex, counterclockwise); level <= 8; no layer_E, no manufactured
   * load.  The host assembly samples the fields on (2^d)^2 elements and rounds the products
   * of the fields with the automata by TT-SVD on the host: about 4 s at level 4 and 80 s at
   * level 5 (the rounding cost grows with the third power of the product ranks). */
  int has_quad;
  double quad[4][2];
  /* Optional heterogeneous material in 2D (Sec. 7, non-homogeneous materials): a weight per
   * element, elem_weight[i * (2^d - 1) + j] for element (i, j) (i along x), positive, that
   * scales the stiffness of that element (E(x) = w E at fixed nu, or w C).  Assembled by
   * the quadrilateral path (a box is the rectangle with corners (0,0), (Lx,0), (0,Ly),
   * (Lx,Ly)): the weighted coefficient fields are compressed to QTT like the Jacobian
   * terms, so any field is accepted (its QTT rank sets the operator's).  2D only, level
   * <= 8, not with layer_E.  Host, n_elem_weight = (2^d - 1)^2 values, copied. */
  int n_elem_weight;
  const double* elem_weight;
} tnfem_problem_desc;

/*
 * Solve options (the AMEn constants; the paper names the solver only).
 * precision: 0 = FP64 everywhere.  1 / 2 = the local CG iterations apply the
 * local operator with FP32 / BF16 operands and FP32 accumulation (MFMA), while
 * interfaces, QR, SVD truncation, enrichment, CG vectors and scalars stay FP64;
 * every local solve is refined: after the low-precision CG stops, the residual is
 * recomputed with the FP64 operator and CG restarts on it until that FP64
 * residual meets the same target as precision 0.  A restart whose FP64
 * residual is not below 0.9 x the best one so far returns to the best iterate
 * and finishes that local solve in FP64 (counted in precision_fallbacks); a
 * low-precision pass stops after 100 iterations.  Operator cores with dense
 * plans (next to the component core) always use FP64.
 */
typedef struct {
  int rank_cap;      /* maximal TT rank of u, 1 .. 252 */
  double tol;        /* stop when every local relative residual <= tol */
  int max_sweeps;    /* half-sweeps (alternating direction) */
  int rho;           /* rank of the residual-projection TT used for enrichment */
  int init_rank;     /* rank of the random initial guess */
  uint64_t seed_x;   /* SplitMix64 seed of the initial guess */
  uint64_t seed_z;   /* SplitMix64 seed of the residual-projection TT */
  int cg_maxit;      /* iteration limit of each local conjugate-gradient solve */
  int precision;
  int profile;       /* 1: time every contraction launch with HIP events (adds host work) */
  /* Outer FP64 iterative refinement (ir_max > 0): the sweeps above give u; then up to ir_max
   * times the same sweep (ir_sweeps half-sweeps, 0 = max_sweeps; a fresh random start of seeds
   * seed_x + i, seed_z + i) solves the correction equation A d = b - A u, whose load b - A u
   * is never formed: its local right-hand sides and residual projections take the FP64 term
   * (left interface) A_k u_k (right interface) with interfaces between the iterate and u
   * through A, built in FP64; then u <- round(u + d) in FP64 on the device (orthogonalisation
   * and SVD truncation at 0.1 ir_tol, ranks at most rank_cap).  Stops once
   * ||d|| <= ir_tol ||u|| (0 = tol).  With ir_max > 0 and precision > 0 a local solve keeps
   * its low-precision pass when that pass lowered the FP64 local residual (one FP64 check, no
   * further restarts: the outer loop carries the FP64 correction), and otherwise returns to
   * its best iterate and finishes in FP64 as without refinement.  Needs rank_cap <= 128. */
  int ir_max;
  int ir_sweeps;
  double ir_tol;
} tnfem_solve_opts;

/* Fills opts with the defaults: cap 32, tol 1e-8, 30 sweeps, rho 4, init rank 2,
 * seeds 1 and 2, 500 CG iterations, FP64, no profiling.  Setting the environment
 * variable TNFEM_VERBOSE=1 prints one line per half-sweep to stderr. */
void tnfem_default_opts(tnfem_solve_opts* opts);

typedef struct {
  int sweeps;             /* half-sweeps done */
  int converged;          /* 1 if max local residual <= tol */
  double final_max_res;   /* max local relative residual of the last half-sweep */
  long long cg_iters;     /* local CG iterations, all cores */
  long long local_applies;/* applications of a local operator */
  double flops;           /* counted floating-point operations of the contractions */
  double seconds;         /* wall time of the solve (device synchronised) */
  int max_rank;           /* max TT rank of u */
  long long refinements;  /* precision > 0: FP64 residual restarts of local solves */
  double low_precision_flops; /* counted flops done with FP32/BF16 operands */
  long long precision_fallbacks; /* precision > 0: local solves finished in FP64 after a restart
                                    that did not lower the FP64 residual */
  double contraction_ms;  /* profile = 1: summed device time of the contraction launches (grouped
                             GEMM and fused local apply, HIP events around each kernel) */
  double contraction_flops; /* profile = 1: algorithmic flops of the launches that did work (CG
                               launches queued after convergence return at once: time, no flops) */
  long long contraction_launches; /* profile = 1: number of timed launches */
  double apply_kernel_ms; /* profile = 1: the same for the fused local-apply kernel alone (the
                             precision of the solve) */
  double apply_kernel_flops;
  long long apply_kernel_launches;
  int peak_rank;          /* largest TT rank of the iterate at any bond during the solve */
  int ir_iters;           /* outer refinement steps done */
  double ir_last_update;  /* ||d|| / ||u|| of the last refinement step */
  int sweeps_total;       /* half-sweeps of all solves (the first and the corrections) */
} tnfem_solve_stats;

/* ---------------------------------------------------------------- context */

/* Creates a context on HIP device `device`.  hip_stream may be NULL (the
 * library creates its own default-priority stream).  Fails with TNFEM_EDEVICE
 * if no device is present. */
int tnfem_ctx_create(tnfem_ctx** out, int device, void* hip_stream);

/* Device allocator hooks (Sec. 8 boundary: PyTorch supplies device memory and streams):
 * alloc(bytes, stream, user) returns device memory on the context's device (NULL fails the
 * call with TNFEM_ENOMEM); free(ptr, stream, user) returns it.  stream is the context's
 * stream.  Every device allocation the context makes (problem plans and loads, solve
 * workspaces, scratch of the primitives) goes through them; the allocation-free entry
 * point's fixed array and the request server's own contexts do not. */
typedef void* (*tnfem_alloc_fn)(size_t bytes, void* stream, void* user);
typedef void (*tnfem_free_fn)(void* ptr, void* stream, void* user);
/* tnfem_ctx_create with allocator hooks (both or neither; NULL = hipMalloc / hipFree).  The
 * hooks and `user` must stay valid until the context and its problems are destroyed. */
int tnfem_ctx_create_ex(tnfem_ctx** out, int device, void* hip_stream, tnfem_alloc_fn alloc, tnfem_free_fn free_fn,
                        void* user);
int tnfem_ctx_destroy(tnfem_ctx* ctx);

/* Message of the last failing call in this thread (static storage). */
const char* tnfem_last_error(void);

/* ---------------------------------------------------------------- problems */

/* Assembles the QTT operator A (with boundary conditions) and load b on the
 * host (Alg. 1 on the Cartesian grid: exact Kronecker factors, no rounding of
 * A) and uploads them to the context's device. */
int tnfem_problem_create(tnfem_ctx* ctx, const tnfem_problem_desc* desc, tnfem_problem** out);
/* Frees the problem's device memory.  Destroy every problem before its context. */
int tnfem_problem_destroy(tnfem_problem* p);

/* Shapes: ncores = d + 1; modes[ncores]; mpo_ranks[ncores + 1]; rhs_ranks[ncores + 1]. */
int tnfem_problem_info(const tnfem_problem* p, int* ncores, int* modes, int* mpo_ranks, int* rhs_ranks);

/* Blocking solve of A u = b (Alg. 2, line 2).  On TNFEM_OK or TNFEM_ENOTCONV
 * *u_out receives the solution TT (caller destroys it) and *stats (if non-NULL)
 * is filled. */
int tnfem_solve(tnfem_problem* p, const tnfem_solve_opts* opts, tnfem_tt** u_out, tnfem_solve_stats* stats);

/* Lockstep solve of n problems (1 <= n <= 16) of the same dimension and level,
 * created in the same context, with one set of options (any opts->precision, no
 * outer refinement (ir_max 0), no profile): every problem takes exactly the steps of
 * tnfem_solve and gets the same result bit for bit, including the FP64 refinement of
 * its low-precision local solves, while the local CG iterations of all problems still
 * iterating are issued as shared launches (one fused local apply per rank class and
 * operand precision, one direction update and one vector update per iteration for
 * the whole batch).  Serving batches of requests of one
 * shape bucket (the request server groups queued requests this way).
 * problems[n] (caller-owned); u_out[n] receives a TT per problem whose status[n]
 * is TNFEM_OK or TNFEM_ENOTCONV (NULL otherwise); stats[n] may be NULL.  Returns
 * TNFEM_OK when the batch ran (per-problem outcomes in status), else the error. */
int tnfem_solve_batch(tnfem_problem* const* problems, int n, const tnfem_solve_opts* opts, tnfem_tt** u_out,
                      tnfem_solve_stats* stats, int* status);

/* ---------------------------------------------------------------- serving
 * A server runs many solves on one device at once.  Requests are queued at
 * submission; each of `slots` worker slots (its own HIP stream) takes the oldest
 * queued request together with the other queued requests of its shape bucket
 * (same dimension, level and solve options, no outer refinement; at most
 * max_batch, default 8),
 * assembles their problems on the host, and uploads and starts them as soon as
 * their device bytes (operator plans, load cores and workspaces, counted before
 * any device allocation) fit in the HBM budget next to the running requests, so requests arriving while others run are admitted as slots and
 * memory free up, and the work of different slots overlaps on the device.  A
 * bucket of several requests runs as one lockstep batch (tnfem_solve_batch:
 * shared launches of the local CG iterations).  Requests share no arithmetic: a
 * result is bit for bit the same alone and in a mix.  Latency is measured from
 * submission to the request's completion.  hbm_budget_bytes = 0 means 80% of
 * the free device memory at creation.  A request larger than the whole budget
 * fails with TNFEM_EBUDGET.  Calls are thread safe. */
typedef struct tnfem_server tnfem_server;
typedef struct {
  int queued, running, peak_running;
  long long completed;
  size_t bytes_in_use, peak_bytes, budget_bytes;
  int peak_batch;              /* largest lockstep batch run so far */
  long long batched_requests;  /* requests that ran in a batch of two or more */
} tnfem_server_state;

int tnfem_server_create(int device, int slots, size_t hbm_budget_bytes, tnfem_server** out);
/* Copies desc and opts (NULL opts: defaults); *ticket identifies the request. */
int tnfem_server_submit(tnfem_server* s, const tnfem_problem_desc* desc, const tnfem_solve_opts* opts,
                        long long* ticket);
/* Result of a request: TNFEM_EBUSY while it is not finished (wait = 0), else the
 * solve's status; on TNFEM_OK / TNFEM_ENOTCONV *u_out receives the solution (caller
 * destroys it).  latency_s = completion - submission.  A ticket is returned once. */
int tnfem_server_poll(tnfem_server* s, long long ticket, int wait, tnfem_tt** u_out, tnfem_solve_stats* stats,
                      double* latency_s);
int tnfem_server_info(tnfem_server* s, tnfem_server_state* info);
/* Largest lockstep batch a slot forms (1 .. 16; 1 turns batching off). */
int tnfem_server_set_max_batch(tnfem_server* s, int max_batch);
/* Stops the workers after their running requests; queued requests are dropped. */
int tnfem_server_destroy(tnfem_server* s);

/* ---------------------------------------------------------------- TT objects */

/* Host TT from caller cores (concatenated row-major cores, doubles). */
int tnfem_tt_create(int ncores, const int* modes, const int* ranks, const double* cores, tnfem_tt** out);
/* ncores; modes[ncores]; ranks[ncores + 1] (any pointer may be NULL). */
int tnfem_tt_shape(const tnfem_tt* t, int* ncores, int* modes, int* ranks);
/* Number of doubles of all cores. */
size_t tnfem_tt_size(const tnfem_tt* t);
/* Copies all cores (concatenated) into dst (host, n >= tnfem_tt_size). */
int tnfem_tt_copy_cores(const tnfem_tt* t, double* dst, size_t n);
/* Entries at multi-indices idx[n][ncores] (host). */
int tnfem_tt_eval(const tnfem_tt* t, const int64_t* idx, size_t n, double* out);
int tnfem_tt_destroy(tnfem_tt* t);
/* Frobenius norm of the TT (host FP64: QR of each unfolding, R carried forward). */
int tnfem_tt_norm(const tnfem_tt* t, double* out);
/* Euclidean inner product <a, b> of two TTs of equal mode sizes (host FP64, contracted core
 * by core from the left).  With the load b of a problem and its solution u, the discrete
 * strain energy is <b, u> / 2 (A u = b, u zero on clamped dofs). */
int tnfem_tt_dot(const tnfem_tt* a, const tnfem_tt* b, double* out);
/* ||a - b|| / ||b|| (||a - b|| if b = 0) for TTs of equal mode sizes, in TT format: the
 * difference is the block TT of ranks r_a + r_b, whose norm is taken as above, so nearly
 * equal TTs do not cancel.  Host FP64; cost O(sum_k n_k (r_a + r_b)^3). */
int tnfem_tt_rel_diff(const tnfem_tt* a, const tnfem_tt* b, double* out);

/* ---------------------------------------------------------------- host assembly export
 * Host-only (no device needed).  Dense copies of the operator's cores, for
 * checking the assembly: core k is [R_k][n][n][R_{k+1}] (output index first).
 * ranks[ncores + 1]; dst receives all cores concatenated (n_doubles >= total). */
int tnfem_export_operator(const tnfem_problem_desc* desc, int* ncores, int* modes, int* ranks,
                          double* dst, size_t n_doubles, size_t* needed);
/* Load TT b (same layout as u). */
int tnfem_export_load(const tnfem_problem_desc* desc, int* ncores, int* modes, int* ranks,
                      double* dst, size_t n_doubles, size_t* needed);

/* ---------------------------------------------------------------- device primitives
 * The sweep's building blocks on caller device buffers, for testing and for
 * callers composing their own sweeps.  All run asynchronously on `stream`.
 *
 * Local operator apply (the hot contraction of every local solve):
 *   y[p][j][t] = sum L[p][b][q] A_k[b][j][i][e] x[q][i][s] Rt[t][e][s]
 * with A_k core k of the problem's operator (reversed = 1: core k of the
 * reversed chain, whose bonds are swapped).  L: [p][R_l][q], x: [q][n][s],
 * Rt: [t][R_r][s], y: [p][n][t], all device, row-major, FP64.
 * Workspace is taken from the context. */
int tnfem_prim_local_apply(tnfem_problem* prob, int k, int reversed, int p, int q, int s, int t,
                           const double* L, const double* x, const double* Rt, double* y, void* stream);

/* The same apply by the fused kernel of the sweep's local CG, with operand
 * precision 0 (FP64), 1 (FP32, FP32 accumulate) or 2 (BF16, FP32 accumulate).
 * Only for cores with a sparse plan (TNFEM_EINVAL otherwise). */
int tnfem_prim_local_apply_ex(tnfem_problem* prob, int k, int reversed, int p, int q, int s, int t, const double* L,
                              const double* x, const double* Rt, double* y, int precision, void* stream);

/* Interface update: Lnew[t][e][s] = sum W[p][j][t] L[p][b][q] A_k[b][j][i][e] X[q][i][s].
 * W: [p][n][t], L: [p][R_l][q], X: [q][n][s], Lnew: [t][R_r][s], device. */
int tnfem_prim_env_update(tnfem_problem* prob, int k, int reversed, int p, int q, int s, int t,
                          const double* W, const double* L, const double* X, double* Lnew, void* stream);

/* Reduced QR factorisation A = Q R of eq. qr (Sec. 4), the step that orthogonalises a core
 * unfolding: Householder QR of the m x n row-major matrix A (device, m >= 1,
 * 1 <= n <= 256); Q (m x c, c = min(m, n)) and R (c x n), device, row-major. */
int tnfem_prim_qr(tnfem_ctx* ctx, int m, int n, const double* A, double* Q, double* R, void* stream);

/* Thin SVD of the m x n row-major matrix A (device, n <= 256, m >= 1; the factorisation
 * behind the TT-SVD truncation of Sec. 4, built on the QR of eq. qr):
 * U (m x c), S (c), Vt (c x n), c = min(m, n), singular values descending.
 * One-sided Jacobi on the R factor of a Householder QR. */
int tnfem_prim_svd(tnfem_ctx* ctx, int m, int n, const double* A, double* U, double* S, double* Vt, void* stream);

/* Allocation-free variant of tnfem_prim_svd, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, kernels and results as tnfem_prim_svd; its
 * workspace (the transposed input, the QR factors, the Jacobi rotations) lives in
 * a fixed array of TNFEM_NOALLOC_SCRATCH_BYTES in device memory, one per device,
 * resolved when the first context on that device is created and held until the
 * process ends.  The call allocates nothing on the device or through any library.
 * A shape whose workspace does not fit, tnfem_prim_svd_noalloc_doubles(m, n) >
 * TNFEM_NOALLOC_SCRATCH_BYTES / 8, fails with TNFEM_EINVAL before anything is
 * launched.  Every call on one device shares that device's array and leaves its
 * contents behind (nothing in it needs to start at zero): calls that overlap on
 * one device (different streams, or threads without ordering) race. */
#define TNFEM_NOALLOC_SCRATCH_BYTES ((size_t)16 << 20)
int tnfem_prim_svd_noalloc(tnfem_ctx* ctx, int m, int n, const double* A, double* U, double* S, double* Vt,
                           void* stream);
/* Doubles of workspace tnfem_prim_svd and tnfem_prim_svd_noalloc use for an m x n input
 * (0 for an invalid shape). */
size_t tnfem_prim_svd_noalloc_doubles(int m, int n);

#ifdef __cplusplus
}
#endif

#endif /* TNFEM_H */
