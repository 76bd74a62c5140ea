// Device kernels of the QTT sweep (gfx950) and their host-side launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/tnfem.h"

namespace tnfem {

// Grouped, strided, coefficient-weighted FP64 GEMM on MFMA:
//   C_g[m][n] = beta * C_g[m][n] + alpha * sum_{t in group g} v_t sum_k A_t[m][k] B_t[k][n]
//   A_t[m][k] = A[a_idx(t) * a_slot + m * a_sm + k * a_sk]
//   B_t[k][n] = B[b_idx(t) * b_slot + k * b_sk + n * b_sn]
//   C_g[m][n] = C[c_idx(g) * c_slot + m * c_sm + n * c_sn]
// grp_beg == nullptr: batched mode, group g has one term with a_idx = b_idx = g.
// grp_c == nullptr: c_idx(g) = g.  t_v == nullptr: v_t = 1.
// skip != nullptr and *skip != 0 at launch time on the device: the kernel does nothing.
struct GemmDesc {
  const double* A = nullptr;
  long a_slot = 0, a_sm = 0, a_sk = 0;
  const double* B = nullptr;
  long b_slot = 0, b_sk = 0, b_sn = 0;
  double* C = nullptr;
  long c_slot = 0, c_sm = 0, c_sn = 0;
  int M = 0, N = 0, K = 0;
  int ngroups = 1;
  const int* grp_beg = nullptr;
  const int* grp_c = nullptr;
  const int* t_a = nullptr;
  const int* t_b = nullptr;
  const double* t_v = nullptr;
  double alpha = 1.0, beta = 0.0;
  const int* skip = nullptr;
  double flops = 0.0;  // algorithmic flops of this launch (2 M N K per term), for profiling
  // Split-K: with a partial buffer, groups with few output tiles split their
  // (term, k) iteration space over several workgroups; partial tiles are summed
  // in a fixed order by a second kernel, so results do not depend on timing.
  int max_terms = 1;           // upper bound of terms per group (host knowledge)
  double* partial = nullptr;   // device buffer for partial tiles
  size_t partial_cap = 0;      // its size in doubles
};

void launch_gemm(const GemmDesc& g, hipStream_t s);
// Independent descriptors (no one writes what another reads) in as few launches as
// their tile classes allow; each result equals that of launch_gemm on its own
// descriptor unless the split-K buffer cannot hold every descriptor's splits.
void launch_gemm_multi(const GemmDesc* ds, int n, hipStream_t s);

// Optional per-launch timing of the contraction kernels (launch_gemm and
// launch_fused_apply) on the calling thread: while a profile is installed, every
// launch is bracketed by HIP events on its stream and tagged with its kind and
// the current tag (the CG iteration it belongs to, -1 outside CG loops).
enum ProfKind { PROF_GEMM = 0, PROF_FUSED = 1, PROF_FUSED_LOW = 2 };
struct GemmProfile {
  std::vector<hipEvent_t> ev;
  std::vector<double> flops;
  std::vector<int> kind, tag;
  std::vector<char> valid;
  size_t used = 0;
  size_t limit = 200000;
  ~GemmProfile();
  void reset() {
    used = 0;
    flops.clear();
    kind.clear();
    tag.clear();
    valid.clear();
  }
  // Waits for the recorded events; total milliseconds and number of the launches of
  // the given kind (-1: all kinds), and the flops of those that did work.
  double total_ms(double* total_flops, int kind = -1, long* launches = nullptr);
};
void set_gemm_profile(GemmProfile* p);
void set_profile_tag(int tag);
size_t profile_mark();
// Marks the launches recorded since `mark` whose tag is >= min_tag as having done
// no work (CG launches queued after convergence, which return at once): their time
// still counts, their flops do not.
void profile_drop_from(size_t mark, int min_tag);
// Default split-K partial buffer for launches of the calling thread whose
// descriptor names none (nullptr: no splitting).
void set_gemm_splitk_buffer(double* p, size_t cap_doubles);

// Device scalars of a local CG solve.
enum CgScal { CG_RZ = 0, CG_PQ, CG_RR, CG_GG, CG_THR2, CG_RES, CG_BETA, CG_NSCAL };
enum CgFlag { CG_DONE = 0, CG_ITERS, CG_MAXIT, CG_COUNTER, CG_NFLAG };
// the flag buffer (8 ints) also holds the initial relative residual as a double at ints
// CG_RES_COPY .. CG_RES_COPY + 1 (written with CG_RES by cg_init2)
constexpr int CG_RES_COPY = 4;

// Local preconditioned CG (block Jacobi over the mode index), one iteration =
// (w = B z), then cg_step (after a fused apply that also formed (z, B z)) or
// cg_reduce_dir + cg_update2:
//   init:   r = g - q (q = B x), z = M^-1 r, p = q_rec = 0; scalars rz, rr, gg;
//           res = ||r|| / ||g||; thr = max(0.1 res, tol/2) ||g||; done = (res <= tol/2) or maxit == 0.
//   dir:    p = z + beta p; q_rec = w + beta q_rec (= B p); pq = p . q_rec.
//   update: x += a p; r -= a q_rec; z = M^-1 r (a = rz / pq); beta = rz_new / rz;
//           done when ||r||^2 <= thr^2 or the iteration limit is reached.
// Every kernel returns at once when done is set.

// Fused local apply for operator cores given as term lists: writes split partial
// tiles part[z][i'][tile][32 x 32] of y = (L x A_k x Rt) x (see kernels.hip).
constexpr int FUSED_MAX_MODES = 8;
struct FusedArgs {
  const double* L = nullptr;
  const double* x = nullptr;
  const double* Rt = nullptr;
  double* partial = nullptr;
  int p = 0, q = 0, s = 0, t = 0, Rl = 0, Rr = 0, n = 0;
  const int* slot_b = nullptr;
  const int* slot_i = nullptr;
  const int* beg = nullptr;
  const int* ta = nullptr;
  const int* tb = nullptr;
  const double* tv = nullptr;
  // the one-pass kernels (ranks <= 64) read per term code = b * 16 + i (the slot's L row
  // index and x mode index) with tb and tv, and the n + 1 list offsets by value
  const int* tc = nullptr;
  int begv[FUSED_MAX_MODES + 1] = {};
  int ksplit = 1, tiles_n = 1, ntiles = 1;
  const int* skip = nullptr;
  // ranks above 64 (two-stage apply): the slot products S[slot] = L_b x_i, nslot slots,
  // fused_stage_elems(f) elements of the operand type in a buffer of stage_bytes bytes
  void* stage = nullptr;
  size_t stage_bytes = 0;
  int nslot = 0;
  // optional (CG, p == q and s == t): each workgroup writes the inner product of x with
  // its partial output tile(s) to dots[fused_dot_index]; their sum is (x, A x)
  double* dots = nullptr;
};
// number of inner-product partials a fused apply with dots writes
int fused_dot_count(const FusedArgs& f);
size_t fused_stage_elems(const FusedArgs& f);
int fused_apply_splits(const FusedArgs& f, int max_terms, size_t cap_doubles);  // needs n, p, q, s, t
// Sets the tile counts of f from its ranks (launch_fused_apply does this itself).
void fused_prepare(FusedArgs& f);
// kernel for a fused apply: all ranks <= 32 (one 32 x 32 tile), <= 64 (one 64 x 64 block
// per workgroup), else the two-stage apply (slot products, then 64 x 64 output tiles)
enum FusedKind { FUSED_32 = 0, FUSED_64 = 1, FUSED_TILED = 2 };
int fused_kind(const FusedArgs& f);

// Shared launches across requests (at most FB_MAX per launch).  The argument
// arrays live in device memory; zoff / boff are prefix sums of each request's
// split count (fused apply) or block count (CG kernels).
constexpr int FB_MAX = 16;
struct FusedBatch {
  const FusedArgs* args = nullptr;  // device array of nreq prepared FusedArgs
  int nreq = 0;
  int zoff[FB_MAX + 1] = {};
  int bpw = 1;  // FUSED_64: the largest fused16_bpw of the requests
};
// 16 x 16 output blocks per wavefront of the rank-64 one-pass apply (FP64 / FP32)
int fused16_bpw(const FusedArgs& f);
// All requests must have the same mode count n and the same fused_kind, FUSED_32 or
// FUSED_64 (the two-stage apply of higher ranks is launched per request).
void launch_fused_apply_batch(const FusedBatch& b, int n, int kind, hipStream_t s, int precision = 0);
// precision: 0 FP64, 1 FP32 operands (FP32 accumulate), 2 BF16 operands (FP32 accumulate)
void launch_fused_apply(FusedArgs f, double flops, hipStream_t s, int precision = 0);
// y = sum of the partial tiles written by launch_fused_apply with the same f.
// y = sum of the split partials of a fused apply; with minus_from, y = minus_from - sum
// (element by element, minus_from may equal y).
void launch_fused_sum(FusedArgs f, double* y, hipStream_t s, const double* minus_from = nullptr);
// the split sums of two applies (partials in separate buffers, no stop flags) in one launch:
// y1 = g1 - A1 x1 (or A1 x1 when g1 is null), y2 likewise
void launch_fused_sum2(FusedArgs f1, double* y1, const double* g1, FusedArgs f2, double* y2, const double* g2,
                       hipStream_t s);

// Local PCG with per-block partial sums (no atomics inside the iteration):
// iteration k = apply (w = B z) -> reduce_dir(k) -> update2(k).
enum { CG_RZ0 = 8, CG_ALPHA0 = 10 };  // scal[CG_RZ0 + k % 2] = r.z, scal[CG_ALPHA0 + k % 2] = alpha of iteration k
// the inner-product partials of the fused apply (cg_step) live at parts + CG_DOT_OFFSET
constexpr int CG_DOT_OFFSET = 4 * 512, CG_DOT_MAX = 1024;
struct CgIterArgs {
  int N = 0;
  double *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
  const double* w = nullptr;        // apply output when ksplit == 0
  const double* partial = nullptr;  // fused-apply partial tiles when ksplit > 0
  int ksplit = 0, n = 0, t = 0, tiles_n = 1, ntiles = 1;
  double* scal = nullptr;
  int* flag = nullptr;
  double* parts = nullptr;  // 5 * 512 doubles
  int maxit = 0;
  int nb_upd = 1;  // blocks of init / update (partials of r.z, r.r)
  int nb_dir = 1;  // blocks of reduce_dir (partials of p.q)
  int keep_thr = 0;  // init: keep the stored threshold (refinement restart) instead of deriving it
  // block-Jacobi preconditioner over the mode index: z[a, :, c] = binv[a, c] r[a, :, c],
  // binv [p][t][bn][bn]; bnp = bn rounded up to a power of two (lanes per block); bt = t
  int bn = 0, bnp = 1, bt = 1;
  const double* binv = nullptr;
  // > 0: the apply wrote ndots partials of (z, B z) at parts + CG_DOT_OFFSET (cg_step)
  int ndots = 0;
  // cg_step launch: nb_step blocks of nt_step (64 or 256) threads, set by cg_step_shape;
  // iteration 0 reads the nb_upd partials of the init kernel, later ones nb_step
  int nb_step = 1, nt_step = 256;
};
int cg_dir_blocks(int n);
void launch_cg_init2(const CgIterArgs& a, const double* g, const double* bx, double tol, hipStream_t s);
void launch_cg_reduce_dir(const CgIterArgs& a, int k, hipStream_t s);
void launch_cg_update2(const CgIterArgs& a, int k, hipStream_t s);
// One kernel per iteration after a fused apply that wrote its (z, B z) partials
// (Chronopoulos-Gear form of the same PCG): replaces reduce_dir + update2.
void launch_cg_step(const CgIterArgs& a, int k, hipStream_t s);
void cg_step_check(const CgIterArgs& a);  // throws unless the arguments fit cg_step
// Sets nb_step / nt_step from N, bn, bnp: one element per thread, 64-thread blocks while
// that needs at most CG_MAXB blocks (the vector work spread over more compute units),
// else 256-thread blocks.
void cg_step_shape(CgIterArgs& a);
struct CgBatch {
  const CgIterArgs* args = nullptr;  // device array
  int nreq = 0;
  int nt = 256;  // step batches: the common nt_step of the requests
  int boff[FB_MAX + 1] = {};
};
void launch_cg_reduce_dir_batch(const CgBatch& b, int k, hipStream_t s);  // boff over nb_dir
void launch_cg_update2_batch(const CgBatch& b, int k, hipStream_t s);     // boff over nb_upd
void launch_cg_step_batch(const CgBatch& b, int k, hipStream_t s);        // boff over nb_upd

// Explicit local matrix of a dense operator core A2 (rows (b, in-index), columns (out-index, e)):
//   Bm[(a n + j) t + c][(a' n + i) t + c'] = sum_{b,e} L[a][b][a'] A[b][j][i][e] Rt[c][e][c'],
// through M[b][j][i][c][c'] = sum_e A[b][j][i][e] Rt[c][e][c'] (Rl n^2 t^2 doubles).
void launch_local_matrix(int p, int n, int t, int Rl, int Rr, const double* L, const double* A2, const double* Rt,
                         double* M, double* Bm, hipStream_t s);
// y = Bm z (N x N row-major); does nothing when skip != nullptr and *skip != 0 on the device.
void launch_dense_matvec(int N, const double* Bm, const double* z, double* y, const int* skip, hipStream_t s);

// Inverses of the diagonal mode blocks of the local operator, for the block-Jacobi
// preconditioner: blk[a, c][j][i] = sum over the operator's nonzero terms (b, j, i, e, v)
// of v L[a][b][a] Rt[c][e][c]; binv[(a t + c) n n + j n + i] = blk[a, c]^{-1}.  Terms grouped
// by mode pair j n + i (beg[n n + 1]; kb = b, ke = e, kv = v).
void launch_local_block_inv(int p, int n, int t, int Rl, int Rr, const double* L, const double* Rt, const int* beg,
                            const int* kb, const int* ke, const double* kv, double* binv, hipStream_t s);

// Householder QR of A (m x n, row-major, lda): Q (m x c), R (c x n), c = min(m, n).
// ws: workspace of ws_cap doubles; throws TNFEM_EINVAL on the host (nothing launched)
// when ws_cap < qr_ws_doubles(m, n), the most any variant may use.
void launch_qr(int m, int n, const double* A, int lda, double* Q, int ldq, double* R, int ldr, double* ws,
               size_t ws_cap, hipStream_t s);

// Batched QR: one workgroup per job, each the same computation as launch_qr.
struct QrJob {
  int m = 0, n = 0, lda = 0, ldq = 0, ldr = 0;
  const double* A = nullptr;
  double *Q = nullptr, *R = nullptr, *ws = nullptr;
  size_t ws_cap = 0;  // doubles at ws; checked against qr_ws_doubles(m, n) before any launch
};
constexpr int QR_BATCH_MAX = 32;
struct QrBatch {
  int njob = 0;
  QrJob job[QR_BATCH_MAX];
};
// Throws TNFEM_EINVAL (nothing launched) when a job's ws_cap is below qr_ws_doubles(m, n).
void launch_qr_batch(const std::vector<QrJob>& jobs, hipStream_t s);
// doubles of ws a QR of an m x n matrix may use (every variant)
size_t qr_ws_doubles(int m, int n);

// One-sided Jacobi SVD of the square n x n matrix G (row-major, ldg): G = U diag(S) V^T,
// S descending.  U, V: n x n row-major.  ws: 3 n (n + 1) doubles (used when n > 64).
// trans != 0: works on G^T (element (i, j) read from G[j * ldg + i]).  U is formed from
// the normalised columns of the rotated matrix, V from the accumulated rotations; for
// the SVD of R^T (trans = 1, R from a QR) the caller passes the destinations swapped:
// U receives R's right and V its left singular vectors.  left_only: only U and S are
// needed; for n <= 64 the rotations are then not accumulated and V is not written.
void launch_jacobi_svd(int n, const double* G, int ldg, double* U, double* S, double* V, double* ws, hipStream_t s,
                       int trans = 0, bool left_only = false);

// Batched Jacobi SVD: one workgroup per job, each the same computation as launch_jacobi_svd.
struct SvdJob {
  int n = 0, ldg = 0;
  const double* G = nullptr;
  double *U = nullptr, *S = nullptr, *V = nullptr, *ws = nullptr;
  int trans = 0;
  bool left_only = false;
};
constexpr int SVD_BATCH_MAX = 16;
struct SvdBatch {
  int njob = 0;
  SvdJob job[SVD_BATCH_MAX];
};
void launch_jacobi_svd_batch(const std::vector<SvdJob>& jobs, hipStream_t s);

// out[0] = smallest r with sum_{j>=r} S_j^2 <= tol^2 sum S^2, clipped to [1, cap].
void launch_trunc_rank(int c, const double* S, double tol, int cap, int* out, hipStream_t s);

// dst[i][j] = alpha * src[i][j] (+ beta * dst) for i < rows, j < cols.
// dst = [src1 | src2] column blocks, row by row (rows x (c1 + c2), leading dimensions given)
void launch_copy_concat(int rows, int c1, const double* src1, long ld1, int c2, const double* src2, long ld2,
                        double* dst, long ldd, hipStream_t s);
void launch_copy2d(int rows, int cols, const double* src, long sld, double* dst, long dld, double alpha, double beta,
                   hipStream_t s);

// W[i][j] = S[i] * V[j][i] for i < r, j < n (V: n x ldv row-major).  Builds diag(S) V^T.
void launch_scale_vt(int r, int n, const double* S, const double* V, int ldv, double* W, hipStream_t s);

// W[i][j] = S[i] * Vt[i][j] for i < r, j < n (Vt row-major, leading dimension ldv).
void launch_scale_rows(int r, int n, const double* S, const double* Vt, int ldv, double* W, hipStream_t s);

// Core transpose for chain reversal: out[b][i][a] = in[a][i][b], in: [ra][n][rb].
void launch_core_transpose(int ra, int n, int rb, const double* in, double* out, hipStream_t s);
// the same for independent (ra, n, rb, in, out) jobs, TRANSPOSE_MULTI_MAX to a launch
struct TransposeJob {
  int ra = 0, n = 0, rb = 0;
  const double* in = nullptr;
  double* out = nullptr;
};
constexpr int TRANSPOSE_MULTI_MAX = 48;
struct TransposeJobs {
  TransposeJob job[TRANSPOSE_MULTI_MAX];
  int beg[TRANSPOSE_MULTI_MAX + 1];
  int n;
};
void launch_core_transpose_multi(const TransposeJob* jobs, int n, hipStream_t s);

// out = a - b (n entries)
void launch_sub(long n, const double* a, const double* b, double* out, hipStream_t s);

// flag[k] = 1 if any of the n values is not finite (OR accumulated).
void launch_nan_check(long n, const double* x, int* flag, hipStream_t s);

// Thin SVD A = U diag(S) Vt of an m x n row-major matrix (c = min(m, n) <= 256): Householder
// QR of the tall orientation, then one-sided Jacobi on R^T.  U: m x c, S: c (descending),
// Vt: c x n, all row-major.  ws holds ws_cap >= svd_ws_doubles(m, n) doubles and needs no
// initial contents (throws TNFEM_EINVAL otherwise, nothing launched).
size_t svd_ws_doubles(int m, int n);
void svd_device(int m, int n, const double* A, double* U, double* S, double* Vt, double* ws, size_t ws_cap,
                hipStream_t st);

// Fixed workspace of the allocation-free entry points: TNFEM_NOALLOC_SCRATCH_BYTES per
// device.  noalloc_init (device current or not) resolves that device's address once;
// noalloc_scratch returns it, or throws TNFEM_EDEVICE when it could not be resolved.
constexpr size_t NOALLOC_SCRATCH_DOUBLES = TNFEM_NOALLOC_SCRATCH_BYTES / sizeof(double);
void noalloc_init(int device);
double* noalloc_scratch(int device);

}  // namespace tnfem
