// C ABI entry points (declared in include/tnfem.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>

#include "assembly.hpp"
#include "common.hpp"
#include "engine.hpp"
#include "hostla.hpp"
#include "kernels.hpp"

struct tnfem_ctx {
  tnfem::Context c;
};
struct tnfem_problem {
  std::unique_ptr<tnfem::Problem> p;
  tnfem_ctx* ctx;
  int device;
};

namespace tnfem {
static thread_local std::string g_last_error;
void set_last_error(const char* msg) { g_last_error = msg ? msg : ""; }
}  // namespace tnfem

using tnfem::fail;

template <class F>
static int guarded(F&& f) {
  try {
    return f();
  } catch (const tnfem::Error& e) {
    tnfem::set_last_error(e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    tnfem::set_last_error("host allocation failed");
    return TNFEM_ENOMEM;
  } catch (const std::exception& e) {
    tnfem::set_last_error(e.what());
    return TNFEM_EINVAL;
  }
}

static hipStream_t pick_stream(tnfem_ctx* ctx, void* s) {
  return s ? static_cast<hipStream_t>(s) : ctx->c.stream;
}

// ----------------------------------------------------------------------------- thin SVD

static void check_svd_args(tnfem_ctx* ctx, int m, int n, const double* A, double* U, double* S, double* Vt) {
  if (!ctx || !A || !U || !S || !Vt) fail(TNFEM_EINVAL, "NULL argument");
  if (m < 1 || n < 1 || std::min(m, n) > 256) fail(TNFEM_EINVAL, "need m, n >= 1 and min(m, n) <= 256");
}

extern "C" {

const char* tnfem_last_error(void) { return tnfem::g_last_error.c_str(); }

void tnfem_default_opts(tnfem_solve_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->rank_cap = 32;
  o->tol = 1e-8;
  o->max_sweeps = 30;
  o->rho = 4;
  o->init_rank = 2;
  o->seed_x = 1;
  o->seed_z = 2;
  o->cg_maxit = 500;
  o->precision = 0;
}

int tnfem_ctx_create(tnfem_ctx** out, int device, void* hip_stream) {
  return tnfem_ctx_create_ex(out, device, hip_stream, nullptr, nullptr, nullptr);
}

int tnfem_ctx_create_ex(tnfem_ctx** out, int device, void* hip_stream, tnfem_alloc_fn alloc, tnfem_free_fn free_fn,
                        void* user) {
  return guarded([&] {
    if ((alloc == nullptr) != (free_fn == nullptr)) fail(TNFEM_EINVAL, "give both allocator hooks or neither");
    if (!out) fail(TNFEM_EINVAL, "out is NULL");
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) fail(TNFEM_EDEVICE, "no HIP device");
    if (device < 0 || device >= count) fail(TNFEM_EINVAL, "device %d out of range (%d devices)", device, count);
    auto c = std::make_unique<tnfem_ctx>();
    c->c.device = device;
    tnfem::hip_check(hipSetDevice(device), "hipSetDevice");
    tnfem::noalloc_init(device);  // fixed workspace of the allocation-free entry points
    if (hip_stream) {
      c->c.stream = static_cast<hipStream_t>(hip_stream);
    } else {
      tnfem::hip_check(hipStreamCreateWithFlags(&c->c.stream, hipStreamNonBlocking), "hipStreamCreate");
      c->c.own_stream = true;
    }
    c->c.allocator.alloc = alloc;
    c->c.allocator.free = free_fn;
    c->c.allocator.user = user;
    c->c.allocator.stream = c->c.stream;
    *out = c.release();
    return TNFEM_OK;
  });
}

int tnfem_ctx_destroy(tnfem_ctx* ctx) {
  return guarded([&] {
    if (!ctx) return TNFEM_OK;
    (void)hipSetDevice(ctx->c.device);
    (void)hipStreamSynchronize(ctx->c.stream);
    ctx->c.allocator.release(ctx->c.scratch);
    ctx->c.allocator.release(ctx->c.splitk);
    if (ctx->c.own_stream) (void)hipStreamDestroy(ctx->c.stream);
    delete ctx;
    return TNFEM_OK;
  });
}

int tnfem_problem_create(tnfem_ctx* ctx, const tnfem_problem_desc* desc, tnfem_problem** out) {
  return guarded([&] {
    if (!ctx || !desc || !out) fail(TNFEM_EINVAL, "NULL argument");
    auto p = std::make_unique<tnfem_problem>();
    p->ctx = ctx;
    p->device = ctx->c.device;
    p->p = tnfem::make_problem(&ctx->c, *desc);
    *out = p.release();
    return TNFEM_OK;
  });
}

int tnfem_problem_destroy(tnfem_problem* p) {
  return guarded([&] {
    if (!p) return TNFEM_OK;
    // the context may already be gone only if the caller broke the documented order;
    // touch nothing of it here (hipFree in the destructors waits for the device)
    (void)hipSetDevice(p->device);
    delete p;
    return TNFEM_OK;
  });
}

int tnfem_problem_info(const tnfem_problem* p, int* ncores, int* modes, int* mpo_ranks, int* rhs_ranks) {
  return guarded([&] {
    if (!p) fail(TNFEM_EINVAL, "NULL problem");
    const auto& P = *p->p;
    if (ncores) *ncores = P.K;
    for (int k = 0; k < P.K; ++k) {
      if (modes) modes[k] = P.modes[k];
    }
    for (int k = 0; k <= P.K; ++k) {
      if (mpo_ranks) mpo_ranks[k] = P.mrank[0][k];
      if (rhs_ranks) rhs_ranks[k] = P.brank[0][k];
    }
    return TNFEM_OK;
  });
}

int tnfem_solve(tnfem_problem* p, const tnfem_solve_opts* opts, tnfem_tt** u_out, tnfem_solve_stats* stats) {
  return guarded([&] {
    if (!p || !u_out) fail(TNFEM_EINVAL, "NULL argument");
    tnfem_solve_opts o;
    if (opts) o = *opts;
    else tnfem_default_opts(&o);
    auto t = std::make_unique<tnfem_tt>();
    tnfem_solve_stats st;
    std::memset(&st, 0, sizeof st);
    const int rc = tnfem::run_solve(*p->p, o, t->t, st);
    if (stats) *stats = st;
    if (rc == TNFEM_OK || rc == TNFEM_ENOTCONV) {
      *u_out = t.release();
    } else {
      *u_out = nullptr;
      tnfem::set_last_error("non-finite value in the sweep");
    }
    if (rc == TNFEM_ENOTCONV) tnfem::set_last_error("sweep limit reached before the tolerance");
    return rc;
  });
}

int tnfem_solve_batch(tnfem_problem* const* problems, int n, const tnfem_solve_opts* opts, tnfem_tt** u_out,
                      tnfem_solve_stats* stats, int* status) {
  return guarded([&] {
    if (!problems || !u_out || !status || n < 1) fail(TNFEM_EINVAL, "NULL argument or empty batch");
    tnfem_solve_opts o;
    if (opts) o = *opts;
    else tnfem_default_opts(&o);
    std::vector<tnfem::Problem*> ps;
    for (int i = 0; i < n; ++i) {
      if (!problems[i]) fail(TNFEM_EINVAL, "NULL problem %d", i);
      ps.push_back(problems[i]->p.get());
    }
    std::vector<tnfem::HostTT> outs;
    std::vector<tnfem_solve_stats> st;
    std::vector<int> rcs;
    tnfem::run_solve_batch(ps, o, outs, st, rcs);
    for (int i = 0; i < n; ++i) {
      status[i] = rcs[i];
      if (stats) stats[i] = st[i];
      u_out[i] = nullptr;
      if (rcs[i] == TNFEM_OK || rcs[i] == TNFEM_ENOTCONV) {
        auto t = std::make_unique<tnfem_tt>();
        t->t = std::move(outs[i]);
        u_out[i] = t.release();
      }
    }
    return TNFEM_OK;
  });
}

int tnfem_tt_create(int ncores, const int* modes, const int* ranks, const double* cores, tnfem_tt** out) {
  return guarded([&] {
    if (ncores < 1 || !modes || !ranks || !cores || !out) fail(TNFEM_EINVAL, "invalid TT description");
    if (ranks[0] != 1 || ranks[ncores] != 1) fail(TNFEM_EINVAL, "boundary ranks must be 1");
    auto t = std::make_unique<tnfem_tt>();
    size_t off = 0;
    for (int k = 0; k < ncores; ++k) {
      if (modes[k] < 1 || ranks[k] < 1 || ranks[k + 1] < 1) fail(TNFEM_EINVAL, "nonpositive mode or rank");
      const size_t cnt = (size_t)ranks[k] * modes[k] * ranks[k + 1];
      t->t.cores.emplace_back(cores + off, cores + off + cnt);
      off += cnt;
    }
    t->t.modes.assign(modes, modes + ncores);
    t->t.ranks.assign(ranks, ranks + ncores + 1);
    *out = t.release();
    return TNFEM_OK;
  });
}

int tnfem_tt_shape(const tnfem_tt* t, int* ncores, int* modes, int* ranks) {
  return guarded([&] {
    if (!t) fail(TNFEM_EINVAL, "NULL TT");
    const int K = (int)t->t.modes.size();
    if (ncores) *ncores = K;
    if (modes) std::copy(t->t.modes.begin(), t->t.modes.end(), modes);
    if (ranks) std::copy(t->t.ranks.begin(), t->t.ranks.end(), ranks);
    return TNFEM_OK;
  });
}

size_t tnfem_tt_size(const tnfem_tt* t) {
  if (!t) return 0;
  size_t s = 0;
  for (const auto& c : t->t.cores) s += c.size();
  return s;
}

int tnfem_tt_copy_cores(const tnfem_tt* t, double* dst, size_t n) {
  return guarded([&] {
    if (!t || !dst) fail(TNFEM_EINVAL, "NULL argument");
    if (n < tnfem_tt_size(t)) fail(TNFEM_EINVAL, "destination too small");
    size_t off = 0;
    for (const auto& c : t->t.cores) {
      std::copy(c.begin(), c.end(), dst + off);
      off += c.size();
    }
    return TNFEM_OK;
  });
}

int tnfem_tt_eval(const tnfem_tt* t, const int64_t* idx, size_t n, double* out) {
  return guarded([&] {
    if (!t || (n && (!idx || !out))) fail(TNFEM_EINVAL, "NULL argument");
    const auto& T = t->t;
    const int K = (int)T.modes.size();
    std::vector<double> v, w;
    for (size_t q = 0; q < n; ++q) {
      v.assign(1, 1.0);
      for (int k = 0; k < K; ++k) {
        const int64_t i = idx[q * K + k];
        if (i < 0 || i >= T.modes[k]) fail(TNFEM_EINVAL, "index out of range");
        const int rl = T.ranks[k], rr = T.ranks[k + 1];
        w.assign(rr, 0.0);
        for (int a = 0; a < rl; ++a)
          for (int b = 0; b < rr; ++b) w[b] += v[a] * T.cores[k][((size_t)a * T.modes[k] + i) * rr + b];
        v.swap(w);
      }
      out[q] = v[0];
    }
    return TNFEM_OK;
  });
}

}  // extern "C"

namespace {

// Frobenius norm of a TT by left-orthogonalisation: QR of each unfolding, the R
// factor carried into the next core; the norm is that of the last carried core.

}  // namespace

extern "C" {

int tnfem_tt_norm(const tnfem_tt* t, double* out) {
  return guarded([&] {
    if (!t || !out) fail(TNFEM_EINVAL, "NULL argument");
    *out = tnfem::hostla::tt_norm(t->t.modes, t->t.ranks, t->t.cores);
    return TNFEM_OK;
  });
}

int tnfem_tt_rel_diff(const tnfem_tt* a, const tnfem_tt* b, double* out) {
  return guarded([&] {
    if (!a || !b || !out) fail(TNFEM_EINVAL, "NULL argument");
    const auto& A = a->t;
    const auto& B = b->t;
    const int K = (int)A.modes.size();
    if (K < 1 || B.modes != A.modes) fail(TNFEM_EINVAL, "TTs have different mode sizes");
    // a - b as a TT of ranks ra + rb: first core [A_0, -B_0], middle block diagonal, last [A; B]
    std::vector<int> ranks(K + 1);
    std::vector<std::vector<double>> cores(K);
    ranks[0] = 1;
    ranks[K] = 1;
    for (int k = 1; k < K; ++k) ranks[k] = A.ranks[k] + B.ranks[k];
    for (int k = 0; k < K; ++k) {
      const int n = A.modes[k];
      const int ral = A.ranks[k], rar = A.ranks[k + 1], rbl = B.ranks[k], rbr = B.ranks[k + 1];
      const int rl = ranks[k], rr = ranks[k + 1];
      cores[k].assign((size_t)rl * n * rr, 0.0);
      const int bl_off = k == 0 ? 0 : ral;       // row offset of B's block
      const int br_off = k == K - 1 ? 0 : rar;   // column offset of B's block
      const double bsign = k == 0 ? -1.0 : 1.0;
      for (int x = 0; x < ral; ++x)
        for (int i = 0; i < n; ++i)
          for (int y = 0; y < rar; ++y)
            cores[k][((size_t)x * n + i) * rr + y] = A.cores[k][((size_t)x * n + i) * rar + y];
      for (int x = 0; x < rbl; ++x)
        for (int i = 0; i < n; ++i)
          for (int y = 0; y < rbr; ++y)
            cores[k][((size_t)(x + bl_off) * n + i) * rr + y + br_off] +=
                bsign * B.cores[k][((size_t)x * n + i) * rbr + y];
    }
    const double nd = tnfem::hostla::tt_norm(A.modes, ranks, std::move(cores));
    const double nb = tnfem::hostla::tt_norm(B.modes, B.ranks, B.cores);
    *out = nb > 0.0 ? nd / nb : nd;
    return TNFEM_OK;
  });
}

int tnfem_tt_dot(const tnfem_tt* a, const tnfem_tt* b, double* out) {
  return guarded([&] {
    if (!a || !b || !out) fail(TNFEM_EINVAL, "NULL argument");
    const auto& A = a->t;
    const auto& B = b->t;
    const int K = (int)A.modes.size();
    if (K < 1 || B.modes != A.modes) fail(TNFEM_EINVAL, "TTs have different mode sizes");
    // left-to-right: E[x][y] = sum over the cores so far of A[.. x] B[.. y]
    std::vector<double> E(1, 1.0);
    for (int k = 0; k < K; ++k) {
      const int n = A.modes[k], ral = A.ranks[k], rar = A.ranks[k + 1], rbl = B.ranks[k], rbr = B.ranks[k + 1];
      // T[x][i][v] = sum_y E[x][y] B[y][i][v]
      std::vector<double> T((size_t)ral * n * rbr, 0.0);
      tnfem::hostla::gemm(ral, n * rbr, rbl, E.data(), B.cores[k].data(), T.data());
      std::vector<double> En((size_t)rar * rbr, 0.0);
      for (int x = 0; x < ral; ++x)
        for (int i = 0; i < n; ++i) {
          const double* arow = &A.cores[k][((size_t)x * n + i) * rar];
          const double* trow = &T[((size_t)x * n + i) * rbr];
          for (int u = 0; u < rar; ++u) {
            const double av = arow[u];
            if (av == 0.0) continue;
            for (int v = 0; v < rbr; ++v) En[(size_t)u * rbr + v] += av * trow[v];
          }
        }
      E.swap(En);
    }
    *out = E[0];
    return TNFEM_OK;
  });
}

int tnfem_tt_destroy(tnfem_tt* t) {
  delete t;
  return TNFEM_OK;
}

int tnfem_export_operator(const tnfem_problem_desc* desc, int* ncores, int* modes, int* ranks, double* dst,
                          size_t n_doubles, size_t* needed) {
  return guarded([&] {
    if (!desc) fail(TNFEM_EINVAL, "NULL descriptor");
    tnfem::Assembled a = tnfem::assemble(*desc);
    const int K = (int)a.A.size();
    size_t tot = 0;
    for (const auto& c : a.A) tot += (size_t)c.Rl * c.n * c.n * c.Rr;
    if (needed) *needed = tot;
    if (ncores) *ncores = K;
    for (int k = 0; k < K; ++k) {
      if (modes) modes[k] = a.A[k].n;
      if (ranks) {
        ranks[k] = a.A[k].Rl;
        ranks[k + 1] = a.A[k].Rr;
      }
    }
    if (dst) {
      if (n_doubles < tot) fail(TNFEM_EINVAL, "destination too small (%zu < %zu)", n_doubles, tot);
      size_t off = 0;
      for (const auto& c : a.A) {
        auto d = c.dense();
        std::copy(d.begin(), d.end(), dst + off);
        off += d.size();
      }
    }
    return TNFEM_OK;
  });
}

int tnfem_export_load(const tnfem_problem_desc* desc, int* ncores, int* modes, int* ranks, double* dst,
                      size_t n_doubles, size_t* needed) {
  return guarded([&] {
    if (!desc) fail(TNFEM_EINVAL, "NULL descriptor");
    tnfem::Assembled a = tnfem::assemble(*desc);
    const int K = (int)a.b.size();
    size_t tot = 0;
    for (const auto& c : a.b) tot += c.data.size();
    if (needed) *needed = tot;
    if (ncores) *ncores = K;
    for (int k = 0; k < K; ++k) {
      if (modes) modes[k] = a.b[k].n;
      if (ranks) {
        ranks[k] = a.b[k].rl;
        ranks[k + 1] = a.b[k].rr;
      }
    }
    if (dst) {
      if (n_doubles < tot) fail(TNFEM_EINVAL, "destination too small");
      size_t off = 0;
      for (const auto& c : a.b) {
        std::copy(c.data.begin(), c.data.end(), dst + off);
        off += c.data.size();
      }
    }
    return TNFEM_OK;
  });
}

int tnfem_prim_local_apply(tnfem_problem* prob, int k, int reversed, int p, int q, int s, int t, const double* L,
                           const double* x, const double* Rt, double* y, void* stream) {
  return guarded([&] {
    if (!prob || !L || !x || !Rt || !y) fail(TNFEM_EINVAL, "NULL argument");
    auto& P = *prob->p;
    if (k < 0 || k >= P.K) fail(TNFEM_EINVAL, "core index %d out of range", k);
    if (p < 1 || q < 1 || s < 1 || t < 1) fail(TNFEM_EINVAL, "ranks must be >= 1");
    tnfem::hip_check(hipSetDevice(prob->ctx->c.device), "hipSetDevice");
    const auto& pl = P.plans[reversed ? 1 : 0][k];
    tnfem::dev_local_apply(P, pl, p, q, s, t, L, x, Rt, y, nullptr, pick_stream(prob->ctx, stream), nullptr);
    return TNFEM_OK;
  });
}

int tnfem_prim_local_apply_ex(tnfem_problem* prob, int k, int reversed, int p, int q, int s, int t, const double* L,
                              const double* x, const double* Rt, double* y, int precision, void* stream) {
  return guarded([&] {
    if (!prob || !L || !x || !Rt || !y) fail(TNFEM_EINVAL, "NULL argument");
    auto& P = *prob->p;
    if (k < 0 || k >= P.K) fail(TNFEM_EINVAL, "core index %d out of range", k);
    if (p < 1 || q < 1 || s < 1 || t < 1) fail(TNFEM_EINVAL, "ranks must be >= 1");
    if (precision < 0 || precision > 2) fail(TNFEM_EINVAL, "precision must be 0, 1 or 2");
    tnfem::hip_check(hipSetDevice(prob->ctx->c.device), "hipSetDevice");
    const auto& pl = P.plans[reversed ? 1 : 0][k];
    tnfem::dev_local_apply_fused(P, pl, p, q, s, t, L, x, Rt, y, precision, pick_stream(prob->ctx, stream));
    return TNFEM_OK;
  });
}

int tnfem_prim_env_update(tnfem_problem* prob, int k, int reversed, int p, int q, int s, int t, const double* W,
                          const double* L, const double* X, double* Lnew, void* stream) {
  return guarded([&] {
    if (!prob || !W || !L || !X || !Lnew) fail(TNFEM_EINVAL, "NULL argument");
    auto& P = *prob->p;
    if (k < 0 || k >= P.K) fail(TNFEM_EINVAL, "core index %d out of range", k);
    if (p < 1 || q < 1 || s < 1 || t < 1) fail(TNFEM_EINVAL, "ranks must be >= 1");
    tnfem::hip_check(hipSetDevice(prob->ctx->c.device), "hipSetDevice");
    const auto& pl = P.plans[reversed ? 1 : 0][k];
    tnfem::dev_env_update(P, pl, p, q, s, t, W, L, X, Lnew, pick_stream(prob->ctx, stream), nullptr);
    return TNFEM_OK;
  });
}

int tnfem_prim_qr(tnfem_ctx* ctx, int m, int n, const double* A, double* Q, double* R, void* stream) {
  return guarded([&] {
    if (!ctx || !A || !Q || !R) fail(TNFEM_EINVAL, "NULL argument");
    if (m < 1 || n < 1 || n > 256) fail(TNFEM_EINVAL, "need m >= 1, 1 <= n <= 256");
    tnfem::hip_check(hipSetDevice(ctx->c.device), "hipSetDevice");
    const int c = std::min(m, n);
    const size_t cap = tnfem::qr_ws_doubles(m, n) + 1;
    double* ws = ctx->c.ensure_scratch(cap);
    tnfem::launch_qr(m, n, A, n, Q, c, R, n, ws, cap, pick_stream(ctx, stream));
    return TNFEM_OK;
  });
}

size_t tnfem_prim_svd_noalloc_doubles(int m, int n) {
  if (m < 1 || n < 1 || std::min(m, n) > 256) return 0;
  return tnfem::svd_ws_doubles(m, n);
}

int tnfem_prim_svd(tnfem_ctx* ctx, int m, int n, const double* A, double* U, double* S, double* Vt, void* stream) {
  return guarded([&] {
    check_svd_args(ctx, m, n, A, U, S, Vt);
    tnfem::hip_check(hipSetDevice(ctx->c.device), "hipSetDevice");
    const size_t need = tnfem::svd_ws_doubles(m, n);
    tnfem::svd_device(m, n, A, U, S, Vt, ctx->c.ensure_scratch(need), need, pick_stream(ctx, stream));
    return TNFEM_OK;
  });
}

int tnfem_prim_svd_noalloc(tnfem_ctx* ctx, int m, int n, const double* A, double* U, double* S, double* Vt,
                           void* stream) {
  return guarded([&] {
    check_svd_args(ctx, m, n, A, U, S, Vt);
    const size_t need = tnfem::svd_ws_doubles(m, n);
    if (need > tnfem::NOALLOC_SCRATCH_DOUBLES)
      fail(TNFEM_EINVAL, "a %d x %d SVD needs %zu doubles of workspace, the fixed workspace holds %zu", m, n, need,
           tnfem::NOALLOC_SCRATCH_DOUBLES);
    tnfem::hip_check(hipSetDevice(ctx->c.device), "hipSetDevice");
    double* ws = tnfem::noalloc_scratch(ctx->c.device);
    tnfem::svd_device(m, n, A, U, S, Vt, ws, need, pick_stream(ctx, stream));
    return TNFEM_OK;
  });
}

}  // extern "C"
