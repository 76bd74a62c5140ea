// The AMEn sweep on the device.
//
// Alg. 2 of the paper applies AMEn (Dolgov and Savostyanov) to A u = M f0.  The
// sweep below follows the published method: alternating half-sweeps over the
// cores; at each core the local system (interfaces x operator core x
// interfaces) is solved by preconditioned conjugate gradients from the current
// core, the solution is truncated by SVD, the basis is enriched with the
// residual projected on a rank-rho residual TT Z, re-orthogonalised by QR, and
// the interfaces are updated.  Every arithmetic step runs in the kernels of
// kernels.hip; the host only sequences launches, reads back the CG status of a
// core and the truncation rank (both needed to size later launches), and
// decides when to stop.  A right-to-left half-sweep is the same code on the
// reversed chain: cores are transposed on the device, operator plans for both
// orientations are built at problem creation.
#include "engine.hpp"
#include "hostla.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>

#include "common.hpp"

namespace tnfem {

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) fail(e == hipErrorOutOfMemory ? TNFEM_ENOMEM : TNFEM_EDEVICE, "%s: %s", what,
                            hipGetErrorString(e));
}

DevArena::~DevArena() { release_all(); }

void DevArena::release_all() {
  for (void* p : ptrs_) {
    if (alloc_) alloc_->release(p);
    else (void)hipFree(p);
  }
  ptrs_.clear();
  bytes_ = 0;
}

void* DeviceAllocator::allocate(size_t bytes) const {
  if (alloc) {
    void* p = alloc(bytes, static_cast<void*>(stream), user);
    if (!p) throw Error(TNFEM_ENOMEM, "the caller's device allocator returned NULL");
    return p;
  }
  void* p = nullptr;
  hip_check(hipMalloc(&p, bytes), "hipMalloc");
  return p;
}

void DeviceAllocator::release(void* p) const {
  if (!p) return;
  if (alloc) {
    if (free) free(p, static_cast<void*>(stream), user);
  } else {
    (void)hipFree(p);
  }
}

void* DevArena::alloc(size_t bytes) {
  if (bytes == 0) bytes = 8;
  if (dry_) {
    bytes_ += bytes;
    return nullptr;
  }
  void* p = alloc_ ? alloc_->allocate(bytes) : nullptr;
  if (!alloc_) hip_check(hipMalloc(&p, bytes), "hipMalloc");
  ptrs_.push_back(p);
  bytes_ += bytes;
  return p;
}

template <class T>
T* DevArena::upload(const std::vector<T>& v, hipStream_t s) {
  T* d = static_cast<T*>(alloc(std::max<size_t>(v.size(), 1) * sizeof(T)));
  if (dry_) return d;
  // blocking copy: callers pass short-lived host vectors (setup only, never in the sweep)
  (void)s;
  if (!v.empty()) hip_check(hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice), "upload");
  return d;
}
template int* DevArena::upload<int>(const std::vector<int>&, hipStream_t);
template double* DevArena::upload<double>(const std::vector<double>&, hipStream_t);

void Context::ensure_splitk() {
  if (!splitk) {
    splitk_cap = (size_t)1 << 22;
    splitk = static_cast<double*>(allocator.allocate(splitk_cap * sizeof(double)));
  }
}

double* Context::ensure_scratch(size_t doubles) {
  if (doubles > scratch_doubles) {
    allocator.release(scratch);
    scratch = nullptr;
    scratch = static_cast<double*>(allocator.allocate(doubles * sizeof(double)));
    scratch_doubles = doubles;
  }
  return scratch;
}

// ----------------------------------------------------------------------------- plans

static MpoCore reversed_core(const MpoCore& c) {
  MpoCore r;
  r.Rl = c.Rr;
  r.Rr = c.Rl;
  r.n = c.n;
  r.b = c.e;
  r.e = c.b;
  r.io = c.io;
  r.ii = c.ii;
  r.v = c.v;
  return r;
}

static Plan build_plan(const MpoCore& c, DevArena& arena, hipStream_t s, size_t* t1_slots, size_t* t2_slots) {
  Plan P;
  P.Rl = c.Rl;
  P.Rr = c.Rr;
  P.n = c.n;
  const int n = c.n;
  // distinct (b, ii) pairs in sorted order
  std::map<std::pair<int, int>, int> slot_of;
  for (size_t t = 0; t < c.nnz(); ++t) slot_of[{c.b[t], c.ii[t]}] = 0;
  const double nnz = (double)c.nnz();
  const double typical_rank = 32.0;
  const double cost_sparse = nnz * typical_rank + (double)slot_of.size() * typical_rank;
  const double cost_dense = (double)c.Rl * n * ((double)n * c.Rr) + (double)n * c.Rr * typical_rank +
                            (double)c.Rl * n * typical_rank;
  P.dense = cost_dense < cost_sparse;
  std::vector<int> sb, si;
  if (P.dense) {
    for (int b = 0; b < c.Rl; ++b)
      for (int i = 0; i < n; ++i) {
        sb.push_back(b);
        si.push_back(i);
      }
  } else {
    int k = 0;
    for (auto& kv : slot_of) {
      kv.second = k++;
      sb.push_back(kv.first.first);
      si.push_back(kv.first.second);
    }
  }
  P.nslot = (int)sb.size();
  std::vector<int> beg(P.nslot + 1);
  for (int i = 0; i <= P.nslot; ++i) beg[i] = i;
  P.slot_beg = arena.upload(beg, s);
  P.slot_b = arena.upload(sb, s);
  P.slot_i = arena.upload(si, s);
  *t1_slots = std::max(*t1_slots, (size_t)P.nslot);

  std::vector<std::vector<int>> ap_a(n), ap_b(n), en_a(c.Rr), en_b(c.Rr);
  std::vector<std::vector<double>> ap_v(n), en_v(c.Rr);
  if (P.dense) {
    std::vector<double> A2((size_t)P.nslot * n * c.Rr, 0.0);
    for (size_t t = 0; t < c.nnz(); ++t)
      A2[((size_t)c.b[t] * n + c.ii[t]) * ((size_t)n * c.Rr) + (size_t)c.io[t] * c.Rr + c.e[t]] += c.v[t];
    P.A2 = arena.upload(A2, s);
    *t2_slots = std::max(*t2_slots, (size_t)n * c.Rr);
    for (int io = 0; io < n; ++io)
      for (int e = 0; e < c.Rr; ++e) {
        ap_a[io].push_back(io * c.Rr + e);
        ap_b[io].push_back(e);
        ap_v[io].push_back(1.0);
        en_a[e].push_back(io);
        en_b[e].push_back(io * c.Rr + e);
        en_v[e].push_back(1.0);
      }
  } else {
    for (size_t t = 0; t < c.nnz(); ++t) {
      const int slot = slot_of[{c.b[t], c.ii[t]}];
      ap_a[c.io[t]].push_back(slot);
      ap_b[c.io[t]].push_back(c.e[t]);
      ap_v[c.io[t]].push_back(c.v[t]);
      en_a[c.e[t]].push_back(c.io[t]);
      en_b[c.e[t]].push_back(slot);
      en_v[c.e[t]].push_back(c.v[t]);
    }
  }
  auto flatten = [&](const std::vector<std::vector<int>>& A, const std::vector<std::vector<int>>& B,
                     const std::vector<std::vector<double>>& V, int** dbeg, int** da, int** db, double** dv,
                     int* gmax) {
    std::vector<int> b0, fa, fb;
    if (gmax) {
      *gmax = 1;
      for (const auto& g : A) *gmax = std::max(*gmax, (int)g.size());
    }
    std::vector<double> fv;
    b0.push_back(0);
    for (size_t g = 0; g < A.size(); ++g) {
      fa.insert(fa.end(), A[g].begin(), A[g].end());
      fb.insert(fb.end(), B[g].begin(), B[g].end());
      fv.insert(fv.end(), V[g].begin(), V[g].end());
      b0.push_back((int)fa.size());
    }
    *dbeg = arena.upload(b0, s);
    *da = arena.upload(fa, s);
    *db = arena.upload(fb, s);
    *dv = arena.upload(fv, s);
    return (int)fa.size();
  };
  P.n_ap = flatten(ap_a, ap_b, ap_v, &P.ap_beg, &P.ap_a, &P.ap_b, &P.ap_v, &P.ap_max);
  P.n_en = flatten(en_a, en_b, en_v, &P.en_beg, &P.en_a, &P.en_b, &P.en_v, &P.en_max);
  // per apply term of the nonzero lists: code = b * 16 + i of its slot (b, i), and the
  // list offsets per output mode on the host
  auto term_codes = [&](const std::vector<std::vector<int>>& A, const std::vector<int>& b_of,
                        const std::vector<int>& i_of) {
    std::vector<int> code, bh{0};
    for (const auto& g : A) {
      for (int slot : g) {
        if (i_of[slot] < 0 || i_of[slot] >= 16) fail(TNFEM_EINVAL, "operator core: mode index beyond 15");
        code.push_back(b_of[slot] * 16 + i_of[slot]);
      }
      bh.push_back((int)code.size());
    }
    P.sp_ap_c = arena.upload(code, s);
    P.sp_beg_h = bh;
  };
  // nonzero term lists (identical to the main lists for sparse plans)
  if (!P.dense) {
    P.sp_nslot = P.nslot;
    P.sp_slot_b = P.slot_b;
    P.sp_slot_i = P.slot_i;
    P.sp_ap_beg = P.ap_beg;
    P.sp_ap_a = P.ap_a;
    P.sp_ap_b = P.ap_b;
    P.sp_ap_v = P.ap_v;
    P.sp_n_ap = P.n_ap;
    P.sp_ap_max = P.ap_max;
    term_codes(ap_a, sb, si);
  } else {
    std::vector<int> ssb, ssi;
    int k2 = 0;
    for (auto& kv : slot_of) {
      kv.second = k2++;
      ssb.push_back(kv.first.first);
      ssi.push_back(kv.first.second);
    }
    P.sp_nslot = (int)ssb.size();
    P.sp_slot_b = arena.upload(ssb, s);
    P.sp_slot_i = arena.upload(ssi, s);
    std::vector<std::vector<int>> sa(n), sbb(n);
    std::vector<std::vector<double>> sv(n);
    for (size_t t = 0; t < c.nnz(); ++t) {
      sa[c.io[t]].push_back(slot_of[{c.b[t], c.ii[t]}]);
      sbb[c.io[t]].push_back(c.e[t]);
      sv[c.io[t]].push_back(c.v[t]);
    }
    P.sp_n_ap = flatten(sa, sbb, sv, &P.sp_ap_beg, &P.sp_ap_a, &P.sp_ap_b, &P.sp_ap_v, &P.sp_ap_max);
    term_codes(sa, ssb, ssi);
  }
  // all terms grouped by (out, in) mode pair: entries of the diagonal mode blocks
  std::vector<std::vector<int>> kb(n * n), ke(n * n);
  std::vector<std::vector<double>> kv(n * n);
  for (size_t t = 0; t < c.nnz(); ++t) {
    const int pr = c.io[t] * n + c.ii[t];
    kb[pr].push_back(c.b[t]);
    ke[pr].push_back(c.e[t]);
    kv[pr].push_back(c.v[t]);
  }
  flatten(kb, ke, kv, &P.bk_beg, &P.bk_b, &P.bk_e, &P.bk_v, nullptr);
  return P;
}

// The fused kernels' view of the nonzero term lists: slot (b, i) resolved per term
// into code = b * 16 + i, and the per-mode list offsets by value.
static void set_terms(FusedArgs& f, const Plan& pl) {
  if (pl.n > FUSED_MAX_MODES || (int)pl.sp_beg_h.size() != pl.n + 1 || !pl.sp_ap_c)
    fail(TNFEM_EINVAL, "fused apply: term lists missing or more than 8 modes");
  f.slot_b = pl.sp_slot_b;
  f.slot_i = pl.sp_slot_i;
  f.beg = pl.sp_ap_beg;
  f.ta = pl.sp_ap_a;
  f.tb = pl.sp_ap_b;
  f.tv = pl.sp_ap_v;
  f.tc = pl.sp_ap_c;
  f.nslot = pl.sp_nslot;
  for (int i = 0; i <= pl.n; ++i) f.begv[i] = pl.sp_beg_h[i];
}

// Builds the plans and load cores of both chain orientations into `arena` (a dry
// arena only counts their bytes).
static void build_device_data(Problem& P, DevArena& arena, hipStream_t s) {
  const auto& A = P.host.A;
  const auto& b = P.host.b;
  P.modes.clear();
  P.maxn = 1;
  P.Rmax = 1;
  P.smax = 1;
  P.t1max_slots = P.t2max_slots = P.sp_slots_max = 1;
  for (int k = 0; k < P.K; ++k) {
    P.modes.push_back(A[k].n);
    P.maxn = std::max(P.maxn, A[k].n);
  }
  for (int o = 0; o < 2; ++o) {
    P.plans[o].clear();
    P.bcore[o].clear();
    P.mrank[o].assign(P.K + 1, 1);
    P.brank[o].assign(P.K + 1, 1);
    for (int j = 0; j < P.K; ++j) {
      const int k = o ? P.K - 1 - j : j;
      MpoCore c = o ? reversed_core(A[k]) : A[k];
      P.plans[o].push_back(build_plan(c, arena, s, &P.t1max_slots, &P.t2max_slots));
      if (!P.plans[o].back().dense) P.sp_slots_max = std::max(P.sp_slots_max, (size_t)P.plans[o].back().sp_nslot);
      P.mrank[o][j] = c.Rl;
      P.mrank[o][j + 1] = c.Rr;
      P.Rmax = std::max(P.Rmax, std::max(c.Rl, c.Rr));
      const TTCore& bc = b[k];
      std::vector<double> data = bc.data;
      int rl = bc.rl, rr = bc.rr;
      if (o) {
        for (int x = 0; x < bc.rl; ++x)
          for (int i = 0; i < bc.n; ++i)
            for (int y = 0; y < bc.rr; ++y) data[((size_t)y * bc.n + i) * bc.rl + x] = bc.data[((size_t)x * bc.n + i) * bc.rr + y];
        std::swap(rl, rr);
      }
      P.bcore[o].push_back(arena.upload(data, s));
      P.brank[o][j] = rl;
      P.brank[o][j + 1] = rr;
      P.smax = std::max(P.smax, std::max(rl, rr));
    }
  }
}

std::unique_ptr<Problem> make_problem_host(const tnfem_problem_desc& desc) {
  auto P = std::make_unique<Problem>();
  P->host = assemble(desc);
  P->K = (int)P->host.A.size();
  DevArena dry(true);
  build_device_data(*P, dry, nullptr);
  P->device_bytes = dry.bytes();
  return P;
}

void upload_problem(Context* ctx, Problem& P) {
  if (P.uploaded) fail(TNFEM_EINVAL, "problem already uploaded");
  P.ctx = ctx;
  hip_check(hipSetDevice(ctx->device), "hipSetDevice");
  P.arena.set_allocator(&ctx->allocator);
  build_device_data(P, P.arena, ctx->stream);
  P.uploaded = true;
  hip_check(hipStreamSynchronize(ctx->stream), "upload sync");
}

std::unique_ptr<Problem> make_problem(Context* ctx, const tnfem_problem_desc& desc) {
  auto P = make_problem_host(desc);
  upload_problem(ctx, *P);
  return P;
}

// ----------------------------------------------------------------------------- contractions

static double flop_count(double m, double n, double k, double terms) { return 2.0 * m * n * k * terms; }

static void count(Flops* f, double m, double n, double k, double terms) {
  if (f) f->total += flop_count(m, n, k, terms);
}

// ---- contraction descriptors (launched alone, or several independent ones at once)

// stage 1 of an apply / interface update: T1[slot] = L_b x_i over the operator's slots
static GemmDesc stage1_desc(const Plan& pl, int p, int q, int s, const double* L, const double* x, const int* skip,
                            double* T1) {
  GemmDesc g1;
  g1.A = L;
  g1.a_slot = q;
  g1.a_sm = (long)pl.Rl * q;
  g1.a_sk = 1;
  g1.B = x;
  g1.b_slot = s;
  g1.b_sk = (long)pl.n * s;
  g1.b_sn = 1;
  g1.C = T1;
  g1.c_slot = (long)p * s;
  g1.c_sm = s;
  g1.c_sn = 1;
  g1.M = p;
  g1.N = s;
  g1.K = q;
  g1.ngroups = pl.nslot;
  g1.grp_beg = pl.slot_beg;
  g1.t_a = pl.slot_b;
  g1.t_b = pl.slot_i;
  g1.skip = skip;
  g1.flops = flop_count(p, s, q, pl.nslot);
  return g1;
}

// dense operator cores: T2 = A2 T1 (the operator core applied to every slot product)
static GemmDesc stage2_dense_desc(const Plan& pl, int p, int s, const double* T1, double* T2, const int* skip) {
  GemmDesc g2;
  g2.A = pl.A2;
  g2.a_sm = 1;
  g2.a_sk = (long)pl.n * pl.Rr;
  g2.B = T1;
  g2.b_sk = (long)p * s;
  g2.b_sn = 1;
  g2.C = T2;
  g2.c_sm = (long)p * s;
  g2.c_sn = 1;
  g2.M = pl.n * pl.Rr;
  g2.N = p * s;
  g2.K = pl.nslot;
  g2.ngroups = 1;
  g2.skip = skip;
  g2.flops = flop_count(g2.M, g2.N, g2.K, 1);
  return g2;
}

// stage 3 of an interface update: Lnew[e] = sum over the terms of e of v W_i^T src
static GemmDesc env_g3_desc(const Plan& pl, int p, int s, int t, const double* W, const double* src, double* Lnew) {
  GemmDesc g3;
  g3.A = W;
  g3.a_slot = t;
  g3.a_sm = 1;
  g3.a_sk = (long)pl.n * t;
  g3.B = src;
  g3.b_slot = (long)p * s;
  g3.b_sk = s;
  g3.b_sn = 1;
  g3.C = Lnew;
  g3.c_slot = s;
  g3.c_sm = (long)pl.Rr * s;
  g3.c_sn = 1;
  g3.M = t;
  g3.N = s;
  g3.K = p;
  g3.ngroups = pl.Rr;
  g3.grp_beg = pl.en_beg;
  g3.t_a = pl.en_a;
  g3.t_b = pl.en_b;
  g3.t_v = pl.en_v;
  g3.max_terms = pl.en_max;
  g3.flops = flop_count(t, s, p, pl.n_en);
  return g3;
}

// Tb[p][n][sb'] = sum Lb[p][sb] B[sb][n][sb'] (first product of the local load and of
// its interface update)
static GemmDesc rhs1_desc(int p, int n, int sb, int sb2, const double* Lb, const double* B, double* Tb) {
  GemmDesc a;
  a.A = Lb;
  a.a_sm = sb;
  a.a_sk = 1;
  a.B = B;
  a.b_sk = (long)n * sb2;
  a.b_sn = 1;
  a.C = Tb;
  a.c_sm = (long)n * sb2;
  a.c_sn = 1;
  a.M = p;
  a.N = n * sb2;
  a.K = sb;
  a.flops = flop_count(p, n * sb2, sb, 1);
  return a;
}

// g[p][n][u] = sum Tb[p][n][sb'] Rb[u][sb']
static GemmDesc rhs2_desc(int p, int n, int sb2, int u, const double* Tb, const double* Rb, double* g) {
  GemmDesc b;
  b.A = Tb;
  b.a_slot = sb2;
  b.a_sm = (long)n * sb2;
  b.a_sk = 1;
  b.B = Rb;
  b.b_slot = 0;
  b.b_sk = 1;
  b.b_sn = sb2;
  b.C = g;
  b.c_slot = u;
  b.c_sm = (long)n * u;
  b.c_sn = 1;
  b.M = p;
  b.N = u;
  b.K = sb2;
  b.ngroups = n;
  b.flops = flop_count(p, u, sb2, n);
  return b;
}

// Lnew[t][sb'] = sum W[p][j][t] Tb[p][j][sb']
static GemmDesc envb2_desc(int p, int n, int sb2, int t, const double* W, const double* Tb, double* Lnew) {
  GemmDesc b;
  b.A = W;
  b.a_sm = 1;
  b.a_sk = t;
  b.B = Tb;
  b.b_sk = sb2;
  b.b_sn = 1;
  b.C = Lnew;
  b.c_sm = sb2;
  b.c_sn = 1;
  b.M = t;
  b.N = sb2;
  b.K = p * n;
  b.flops = flop_count(t, sb2, p * n, 1);
  return b;
}

// C (m x n) = A (m x k) B (k x n), plain row-major (lda/ldb/ldc given); transA reads A^T stored k x m.
static GemmDesc plain_desc(int m, int n, int k, const double* A, long lda, bool transA, const double* B, long ldb,
                           double* C, long ldc) {
  GemmDesc g;
  g.A = A;
  if (transA) {
    g.a_sm = 1;
    g.a_sk = lda;
  } else {
    g.a_sm = lda;
    g.a_sk = 1;
  }
  g.B = B;
  g.b_sk = ldb;
  g.b_sn = 1;
  g.C = C;
  g.c_sm = ldc;
  g.c_sn = 1;
  g.M = m;
  g.N = n;
  g.K = k;
  g.flops = flop_count(m, n, k, 1);
  return g;
}

static void run(const GemmDesc& d, hipStream_t st, Flops* f) {
  launch_gemm(d, st);
  if (f) f->total += d.flops;
}

// Independent contractions issued together (launch_gemm_multi), their flops counted.
struct GemmSet {
  static constexpr int kMax = 8;
  GemmDesc d[kMax];
  int n = 0;
  void add(const GemmDesc& g) {
    if (n == kMax) fail(TNFEM_EINVAL, "contraction set full");
    d[n++] = g;
  }
  void launch(hipStream_t st, Flops* f) {
    launch_gemm_multi(d, n, st);
    if (f)
      for (int i = 0; i < n; ++i) f->total += d[i].flops;
    n = 0;
  }
};

static void stage12(Problem& P, const Plan& pl, int p, int q, int s, const double* L, const double* x, const int* skip,
                    hipStream_t st, Flops* f, double* T1, double* T2, const double** src) {
  run(stage1_desc(pl, p, q, s, L, x, skip, T1), st, f);
  *src = T1;
  if (pl.dense) {
    run(stage2_dense_desc(pl, p, s, T1, T2, skip), st, f);
    *src = T2;
  }
  (void)P;
}

static void local_apply_ws(Problem& P, const Plan& pl, int p, int q, int s, int t, const double* L, const double* x,
                           const double* Rt, double* y, const int* skip, hipStream_t st, Flops* f, double* T1,
                           double* T2) {
  const double* src = nullptr;
  stage12(P, pl, p, q, s, L, x, skip, st, f, T1, T2, &src);
  GemmDesc g3;
  g3.A = src;
  g3.a_slot = (long)p * s;
  g3.a_sm = s;
  g3.a_sk = 1;
  g3.B = Rt;
  g3.b_slot = s;
  g3.b_sk = 1;
  g3.b_sn = (long)pl.Rr * s;
  g3.C = y;
  g3.c_slot = t;
  g3.c_sm = (long)pl.n * t;
  g3.c_sn = 1;
  g3.M = p;
  g3.N = t;
  g3.K = s;
  g3.ngroups = pl.n;
  g3.grp_beg = pl.ap_beg;
  g3.t_a = pl.ap_a;
  g3.t_b = pl.ap_b;
  g3.t_v = pl.ap_v;
  g3.max_terms = pl.ap_max;
  g3.skip = skip;
  g3.flops = flop_count(p, t, s, pl.n_ap);
  run(g3, st, f);
}

static void env_update_ws(Problem& P, const Plan& pl, int p, int q, int s, int t, const double* W, const double* L,
                          const double* X, double* Lnew, hipStream_t st, Flops* f, double* T1, double* T2) {
  const double* src = nullptr;
  stage12(P, pl, p, q, s, L, X, nullptr, st, f, T1, T2, &src);
  run(env_g3_desc(pl, p, s, t, W, src, Lnew), st, f);
}

struct SplitkScope {
  explicit SplitkScope(double* p, size_t cap) { set_gemm_splitk_buffer(p, cap); }
  ~SplitkScope() { set_gemm_splitk_buffer(nullptr, 0); }
};

void dev_local_apply(Problem& P, const Plan& pl, int p, int q, int s, int t, const double* L, const double* x,
                     const double* Rt, double* y, const int* skip, hipStream_t st, Flops* f) {
  const size_t n1 = (size_t)pl.n_t1() * p * s, n2 = (size_t)pl.n_t2() * p * s;
  double* T1 = P.ctx->ensure_scratch(n1 + n2 + 1);
  P.ctx->ensure_splitk();
  SplitkScope sk(P.ctx->splitk, P.ctx->splitk_cap);
  local_apply_ws(P, pl, p, q, s, t, L, x, Rt, y, skip, st, f, T1, T1 + n1);
}

void dev_local_apply_fused(Problem& P, const Plan& pl, int p, int q, int s, int t, const double* L, const double* x,
                           const double* Rt, double* y, int precision, hipStream_t st) {
  if (pl.dense) fail(TNFEM_EINVAL, "this operator core has a dense plan; the fused apply is for sparse plans");
  P.ctx->ensure_splitk();
  FusedArgs f;
  f.L = L;
  f.x = x;
  f.Rt = Rt;
  f.partial = P.ctx->splitk;
  f.p = p;
  f.q = q;
  f.s = s;
  f.t = t;
  f.Rl = pl.Rl;
  f.Rr = pl.Rr;
  f.n = pl.n;
  set_terms(f, pl);
  if (fused_kind(f) == FUSED_TILED) {
    const size_t elems = fused_stage_elems(f);
    f.stage = P.ctx->ensure_scratch(elems);
    f.stage_bytes = elems * sizeof(double);
  }
  f.ksplit = fused_apply_splits(f, pl.sp_ap_max, P.ctx->splitk_cap);
  launch_fused_apply(f, 0.0, st, precision);
  launch_fused_sum(f, y, st);
}

void dev_env_update(Problem& P, const Plan& pl, int p, int q, int s, int t, const double* W, const double* L,
                    const double* X, double* Lnew, hipStream_t st, Flops* f) {
  const size_t n1 = (size_t)pl.n_t1() * p * s, n2 = (size_t)pl.n_t2() * p * s;
  double* T1 = P.ctx->ensure_scratch(n1 + n2 + 1);
  P.ctx->ensure_splitk();
  SplitkScope sk(P.ctx->splitk, P.ctx->splitk_cap);
  env_update_ws(P, pl, p, q, s, t, W, L, X, Lnew, st, f, T1, T1 + n1);
}

// g[p][n][u] = sum Lb[p][sb] B[sb][n][sb'] Rb[u][sb']
static void local_rhs(int p, int n, int sb, int sb2, int u, const double* Lb, const double* B, const double* Rb,
                      double* Tb, double* g, hipStream_t st, Flops* f) {
  run(rhs1_desc(p, n, sb, sb2, Lb, B, Tb), st, f);
  run(rhs2_desc(p, n, sb2, u, Tb, Rb, g), st, f);
}

static void gemm_plain(int m, int n, int k, const double* A, long lda, bool transA, const double* B, long ldb,
                       double* C, long ldc, hipStream_t st, Flops* f) {
  run(plain_desc(m, n, k, A, lda, transA, B, ldb, C, ldc), st, f);
}

// ----------------------------------------------------------------------------- workspace

// Lays out the workspace of a problem for (cap, rho); `A` returns a buffer of the
// given number of doubles (or counts them when only the size is wanted).
// Local systems of dense-plan cores with at most this many unknowns are solved with
// the explicit local matrix (formed once per local solve) instead of the contraction chain.
constexpr size_t kExplicitMaxN = 2048;

template <class Alloc>
static void layout_workspace(const Problem& P, Workspace& W, int cap, int rho, Alloc A) {
  const int K = P.K;
  const size_t maxn = (size_t)P.maxn, Rmax = (size_t)P.Rmax, smax = (size_t)P.smax;
  const size_t rc = (size_t)std::max(cap, rho);
  const size_t core = rc * maxn * rc;
  const size_t zcore = (size_t)rho * maxn * rho;
  const size_t M = rc * maxn, Nw = rc + rho;
  W.X.clear();
  W.Z.clear();
  W.Xalt.clear();
  W.Zalt.clear();
  W.EA.clear();
  W.Eb.clear();
  W.EzA.clear();
  W.Ezb.clear();
  for (int k = 0; k < K; ++k) {
    W.X.push_back(A(core));
    W.Z.push_back(A(std::max(zcore, core)));
    W.Xalt.push_back(A(core));
    W.Zalt.push_back(A(std::max(zcore, core)));
  }
  W.Xspare = A(core);
  W.Zspare = A(std::max(zcore, core));
  for (int k = 0; k <= K; ++k) {
    W.EA.push_back(A(rc * Rmax * rc));
    W.Eb.push_back(A(rc * smax));
    W.EzA.push_back(A((size_t)rho * Rmax * rc));
    W.Ezb.push_back(A((size_t)rho * smax));
  }
  W.T1 = A(P.t1max_slots * rc * rc);
  W.T2 = A(P.t2max_slots * rc * rc);
  W.T1z = A(P.t1max_slots * (size_t)rho * rc);
  W.T2z = A(P.t2max_slots * (size_t)rho * rc);
  W.Tbz = A((size_t)rho * maxn * smax);
  W.g = A(core);
  W.r = A(core);
  W.z = A(core);
  W.p = A(core);
  W.q = A(core);
  W.w = A(core);
  W.binv = A(rc * rc * maxn * maxn);
  W.Tb = A(rc * maxn * smax);
  W.gz = A(core);
  W.yz = A(core);
  W.ge = A(core);
  W.ye = A(core);
  W.Qx = A(M * Nw);
  W.Rx = A(Nw * Nw);
  W.UR = A(Nw * Nw);
  W.S = A(Nw);
  W.V = A(Nw * Nw);
  W.Ur = A(M * Nw);
  W.SVt = A(Nw * Nw);
  W.xT = A(M * Nw);
  W.xt = A(M * Nw);
  W.aug = A(M * Nw);
  W.Qa = A(M * Nw);
  W.Ra = A(Nw * Nw);
  W.Wm = A(Nw * Nw);
  W.qrws_cap = std::max(M * Nw * 2 + 4 * Nw + 2 * Nw * Nw, qr_ws_doubles((int)M, (int)Nw));
  W.qrws = A(W.qrws_cap);
  W.Rz = A((size_t)rho * maxn * rho + 1);
  // residual-TT QR: (rho n) x rho at most, routed to any variant (the blocked one included)
  W.qrwsz_cap = std::max(2 * (size_t)rho * maxn * rho + 4 * (size_t)rho, qr_ws_doubles((int)(rho * maxn), rho));
  W.qrwsz = A(W.qrwsz_cap);
  W.scal = A(16);
  W.fpart_cap = (size_t)1 << 22;
  W.fpart = A(W.fpart_cap);
  if (rc > 64) {  // the two-stage fused apply holds one padded p x s product per slot
    const size_t rc64 = (rc + 63) / 64 * 64;
    W.stage_bytes = P.sp_slots_max * rc64 * rc64 * sizeof(double);
    W.stage = A(P.sp_slots_max * rc64 * rc64);
  } else {
    W.stage_bytes = 0;
    W.stage = nullptr;
  }
  W.splitk_cap = (size_t)1 << 22;
  W.splitk = A(W.splitk_cap);
  W.part = A(6 * 512);
  W.bloc_n = std::min<size_t>(kExplicitMaxN, rc * maxn * rc);
  W.Bloc = A(W.bloc_n * W.bloc_n);
  W.mloc_cap = W.bloc_n * W.bloc_n;
  W.Mloc = A(W.mloc_cap);
}

size_t Problem::workspace_bytes(int cap, int rho) const {
  Workspace W;
  size_t total = 0;
  layout_workspace(*this, W, cap, rho, [&](size_t d) {
    total += std::max<size_t>(d, 1) * 8;
    return static_cast<double*>(nullptr);
  });
  return total + 64 + 4096;
}

void Problem::ensure_workspace(int cap, int rho) {
  if (ws && ws->cap >= cap && ws->rho >= rho) return;
  ws.reset();
  auto W = std::make_unique<Workspace>();
  W->cap = cap;
  W->rho = rho;
  W->arena.set_allocator(&ctx->allocator);
  layout_workspace(*this, *W, cap, rho,
                   [&](size_t d) { return static_cast<double*>(W->arena.alloc(std::max<size_t>(d, 1) * 8)); });
  W->flag = static_cast<int*>(W->arena.alloc(sizeof(int) * 8));
  W->drank = static_cast<int*>(W->arena.alloc(sizeof(int) * 8));
  hip_check(hipMemset(W->flag, 0, sizeof(int) * 8), "memset flag");
  hip_check(hipHostMalloc(&W->host_pinned, 4096, hipHostMallocDefault), "hipHostMalloc");
  ws = std::move(W);
}

void Problem::ensure_ir(int cap, int rho) {
  if (ws->ir && ws->ir->cap >= cap && ws->ir->rho >= rho) return;
  ws->ir.reset();
  auto B = std::make_unique<IrBuffers>();
  B->cap = cap;
  B->rho = rho;
  B->arena.set_allocator(&ctx->allocator);
  auto A = [&](size_t d) { return static_cast<double*>(B->arena.alloc(std::max<size_t>(d, 1) * 8)); };
  const size_t rc = (size_t)std::max(cap, rho), mx = (size_t)maxn, R = (size_t)Rmax;
  const size_t core = rc * mx * rc, r2 = 2 * rc;
  B->sum_cap = r2 * mx * r2;
  for (int k = 0; k < K; ++k) {
    B->U.push_back(A(core));
    B->Sum.push_back(A(B->sum_cap));
  }
  B->uspare = A(core);
  for (int k = 0; k <= K; ++k) {
    B->EuA.push_back(A(rc * R * rc));
    B->EzuA.push_back(A((size_t)rho * R * rc));
  }
  B->t1 = A(B->sum_cap);
  B->t2 = A(B->sum_cap);
  B->su = A(B->sum_cap);
  B->ss = A(r2);
  B->svt = A(r2 * r2);
  B->svdws_cap = svd_ws_doubles((int)(r2 * mx), (int)r2);
  B->svdws = A(B->svdws_cap);
  ws->ir = std::move(B);
}

// ----------------------------------------------------------------------------- SplitMix64

static inline uint64_t splitmix64_at(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static std::vector<std::vector<double>> random_tt_host(const std::vector<int>& modes, int rank, uint64_t seed,
                                                       std::vector<int>& ranks) {
  const int K = (int)modes.size();
  ranks.assign(K + 1, 1);
  for (int k = 1; k < K; ++k) {
    double left = 1, right = 1;
    for (int j = 0; j < k; ++j) left *= modes[j];
    for (int j = k; j < K; ++j) right *= modes[j];
    ranks[k] = (int)std::min<double>(rank, std::min(left, right));
  }
  std::vector<std::vector<double>> cores(K);
  uint64_t off = 0;
  for (int k = 0; k < K; ++k) {
    const size_t cnt = (size_t)ranks[k] * modes[k] * ranks[k + 1];
    cores[k].resize(cnt);
    for (size_t i = 0; i < cnt; ++i) {
      const uint64_t z = splitmix64_at(seed, off + i);
      cores[k][i] = 2.0 * (double)(z >> 11) * (1.0 / 9007199254740992.0) - 1.0;
    }
    off += cnt;
  }
  return cores;
}

// ----------------------------------------------------------------------------- the sweep

namespace {

// Block-Jacobi preconditioner over the mode index: blocks of n unknowns (a, :, c).
static void set_block_precond(CgIterArgs& a, int n, int t, const double* binv) {
  int np2 = 1;
  while (np2 < n) np2 *= 2;
  a.bn = n;
  a.bnp = np2;
  a.bt = t;
  a.binv = binv;
}

struct Sweep {
  Problem& P;
  Workspace& W;
  tnfem_solve_opts o;
  hipStream_t st;
  int K;
  int orient = 0;  // 0: forward chain, 1: reversed
  std::vector<double*> X, Z, EA, Eb, EzA, Ezb;
  std::vector<int> xr, zr;  // K + 1 ranks (current orientation)
  std::vector<int> n;       // modes (current orientation)
  double *xspare = nullptr, *zspare = nullptr;
  std::vector<double*> Xalt, Zalt;
  Flops fl;
  double fl_low = 0.0;
  long long cg_iters = 0, applies = 0, refinements = 0, fallbacks = 0;
  double max_res = 0.0;
  int peak_rank = 0;  // largest rank of u at any bond during the solve
  int nan_seen = 0;
  int verbose = 0;  // 2: one line per local solve on stderr
  std::vector<int> cg_last;  // CG iterations of the last local solve at each core (chain order)
  // outer refinement: the load is b - A u for a fixed TT u (cores U, ranks ur); EuA / EzuA are
  // the interfaces X-A-u and Z-A-u.  ir_inner: low-precision local solves end after their
  // low-precision pass (the outer loop carries the FP64 correction).
  bool with_u = false, ir_inner = false;
  // W.Tb holds Eb[tb_k] B(tb_k), W.Tbz holds Ezb[tbz_k] B(tbz_k) (-1: neither is known);
  // the first product of the local load is reused by the enrichment load and by the
  // interface update of the same core
  int tb_k = -1, tbz_k = -1;
  std::vector<double*> U, EuA, EzuA;
  std::vector<int> ur;
  double* uspare = nullptr;

  Sweep(Problem& p, const tnfem_solve_opts& opts) : P(p), W(*p.ws), o(opts), st(p.ctx->stream), K(p.K) {
    const char* v = std::getenv("TNFEM_VERBOSE");
    verbose = v ? std::atoi(v) : 0;
    cg_last.assign(K, 0);
  }

  volatile int* hint() { return static_cast<volatile int*>(W.host_pinned); }

  void sync() { hip_check(hipStreamSynchronize(st), "hipStreamSynchronize"); }

  void upload_initial() { upload_initial(o.seed_x, o.seed_z); }

  void upload_initial(uint64_t seed_x, uint64_t seed_z) {
    std::vector<int> rx, rz;
    auto cx = random_tt_host(P.modes, o.init_rank, seed_x, rx);
    auto cz = random_tt_host(P.modes, o.rho, seed_z, rz);
    X = W.X;
    Z = W.Z;
    xspare = W.Xspare;
    zspare = W.Zspare;
    Xalt = W.Xalt;
    Zalt = W.Zalt;
    EA = W.EA;
    Eb = W.Eb;
    EzA = W.EzA;
    Ezb = W.Ezb;
    xr = rx;
    zr = rz;
    n = P.modes;
    for (int k = 0; k < K; ++k) {
      hip_check(hipMemcpyAsync(X[k], cx[k].data(), cx[k].size() * 8, hipMemcpyHostToDevice, st), "upload X0");
      hip_check(hipMemcpyAsync(Z[k], cz[k].data(), cz[k].size() * 8, hipMemcpyHostToDevice, st), "upload Z0");
    }
    const double one = 1.0;
    for (double* b : {EA[0], Eb[0], EzA[0], Ezb[0], EA[K], Eb[K], EzA[K], Ezb[K]})
      hip_check(hipMemcpyAsync(b, &one, 8, hipMemcpyHostToDevice, st), "boundary interface");
    if (with_u)
      for (double* b : {EuA[0], EzuA[0], EuA[K], EzuA[K]})
        hip_check(hipMemcpyAsync(b, &one, 8, hipMemcpyHostToDevice, st), "boundary interface");
    sync();  // `one` is on the host stack
  }

  void reverse() {
    tb_k = tbz_k = -1;
    std::vector<TransposeJob> jobs;
    for (int k = 0; k < K; ++k) {
      jobs.push_back(TransposeJob{xr[k], n[k], xr[k + 1], X[k], Xalt[k]});
      jobs.push_back(TransposeJob{zr[k], n[k], zr[k + 1], Z[k], Zalt[k]});
    }
    launch_core_transpose_multi(jobs.data(), (int)jobs.size(), st);
    std::swap(X, Xalt);
    std::swap(Z, Zalt);
    if (with_u) {
      for (int k = 0; k < K; ++k) {
        launch_core_transpose(ur[k], n[k], ur[k + 1], U[k], uspare, st);
        std::swap(U[k], uspare);
      }
      std::reverse(U.begin(), U.end());
      std::reverse(ur.begin(), ur.end());
      std::reverse(EuA.begin(), EuA.end());
      std::reverse(EzuA.begin(), EzuA.end());
    }
    std::reverse(X.begin(), X.end());
    std::reverse(Z.begin(), Z.end());
    std::reverse(xr.begin(), xr.end());
    std::reverse(zr.begin(), zr.end());
    std::reverse(n.begin(), n.end());
    std::reverse(EA.begin(), EA.end());
    std::reverse(Eb.begin(), Eb.end());
    std::reverse(EzA.begin(), EzA.end());
    std::reverse(Ezb.begin(), Ezb.end());
    orient ^= 1;
  }

  const Plan& plan(int k) const { return P.plans[orient][k]; }
  int R(int j) const { return P.mrank[orient][j]; }
  int sb(int j) const { return P.brank[orient][j]; }
  const double* B(int k) const { return P.bcore[orient][k]; }

  // y = local operator applied to x between interfaces L and Rt: the fused kernel plus
  // the ordered sum of its partial tiles for sparse plans, the GEMM chain for dense ones
  // y = A x on the interfaces L, Rt; with minus_from (sparse plans), y = minus_from - A x
  void apply(int k, int p, int q, int s, int t, const double* L, const double* x, const double* Rt, double* y,
             const int* skip, const double* minus_from = nullptr) {
    const Plan& pl = plan(k);
    if (pl.dense) {
      if (minus_from) fail(TNFEM_EINVAL, "apply: subtraction needs a sparse plan");
      local_apply_ws(P, pl, p, q, s, t, L, x, Rt, y, skip, st, &fl, W.T1, W.T2);
      return;
    }
    FusedArgs f = fused_args(k, p, q, s, t, L, x, Rt, W.fpart, W.fpart_cap);
    f.skip = skip;
    const double flops = 2.0 * p * q * s * pl.sp_nslot + 2.0 * p * s * t * pl.sp_n_ap;
    launch_fused_apply(f, flops, st, 0);
    launch_fused_sum(f, y, st, minus_from);
    fl.total += flops;
  }

  // The fused apply of core k's sparse plan on the given interfaces, its split partials in
  // `partial` (cap doubles)
  FusedArgs fused_args(int k, int p, int q, int s, int t, const double* L, const double* x, const double* Rt,
                       double* partial, size_t cap) {
    const Plan& pl = plan(k);
    FusedArgs f;
    f.L = L;
    f.x = x;
    f.Rt = Rt;
    f.partial = partial;
    f.p = p;
    f.q = q;
    f.s = s;
    f.t = t;
    f.Rl = pl.Rl;
    f.Rr = pl.Rr;
    f.n = pl.n;
    set_terms(f, pl);
    f.stage = W.stage;
    f.stage_bytes = W.stage_bytes;
    f.ksplit = fused_apply_splits(f, pl.sp_ap_max, cap);
    return f;
  }

  // g -= A x (tmp holds A x where the plan is dense)
  void apply_sub(int k, int p, int q, int s, int t, const double* L, const double* x, const double* Rt, double* g,
                 double* tmp) {
    if (plan(k).dense) {
      apply(k, p, q, s, t, L, x, Rt, tmp, nullptr);
      launch_sub((long)p * n[k] * t, g, tmp, g, st);
    } else {
      apply(k, p, q, s, t, L, x, Rt, g, nullptr, g);
    }
  }

  // Interfaces at bond k + 1 from core k: the X and Z interface updates (operator and
  // load) are independent, so their stages run as shared launches; pre1 / pre2 are
  // independent products of the caller issued with the first / last stage.
  void update_envs(int k, const GemmDesc* pre1 = nullptr, const GemmDesc* pre2 = nullptr) {
    const int p = xr[k], s = xr[k + 1], pz = zr[k], tz = zr[k + 1];
    const Plan& pl = plan(k);
    GemmSet g;
    if (pre1) g.add(*pre1);
    g.add(stage1_desc(pl, p, p, s, EA[k], X[k], nullptr, W.T1));
    g.add(stage1_desc(pl, pz, p, s, EzA[k], X[k], nullptr, W.T1z));
    if (tb_k != k) g.add(rhs1_desc(p, n[k], sb(k), sb(k + 1), Eb[k], B(k), W.Tb));
    if (tbz_k != k) g.add(rhs1_desc(pz, n[k], sb(k), sb(k + 1), Ezb[k], B(k), W.Tbz));
    g.launch(st, &fl);
    tb_k = tbz_k = k;
    const double *src = W.T1, *srcz = W.T1z;
    if (pl.dense) {
      g.add(stage2_dense_desc(pl, p, s, W.T1, W.T2, nullptr));
      g.add(stage2_dense_desc(pl, pz, s, W.T1z, W.T2z, nullptr));
      g.launch(st, &fl);
      src = W.T2;
      srcz = W.T2z;
    }
    if (pre2) g.add(*pre2);
    g.add(env_g3_desc(pl, p, s, s, X[k], src, EA[k + 1]));
    g.add(envb2_desc(p, n[k], sb(k + 1), s, X[k], W.Tb, Eb[k + 1]));
    g.add(env_g3_desc(pl, pz, s, tz, Z[k], srcz, EzA[k + 1]));
    g.add(envb2_desc(pz, n[k], sb(k + 1), tz, Z[k], W.Tbz, Ezb[k + 1]));
    g.launch(st, &fl);
    if (with_u) {
      const int q = ur[k], s2 = ur[k + 1];
      env_update_ws(P, plan(k), p, q, s2, s, X[k], EuA[k], U[k], EuA[k + 1], st, &fl, W.T1, W.T2);
      env_update_ws(P, plan(k), pz, q, s2, tz, Z[k], EzuA[k], U[k], EzuA[k + 1], st, &fl, W.T1, W.T2);
    }
  }

  // Left-orthogonalise core k of T (ranks tr) by QR and carry R into core k+1.
  void qr_step(std::vector<double*>& T, std::vector<int>& tr, int k, double* spare) {
    const int m = tr[k] * n[k], nc = tr[k + 1];
    const int c = std::min(m, nc);
    launch_qr(m, nc, T[k], nc, W.Qa, c, W.Ra, nc, W.qrws, W.qrws_cap, st);
    launch_copy2d(m, c, W.Qa, c, T[k], c, 1.0, 0.0, st);
    const int cols = n[k + 1] * tr[k + 2];
    gemm_plain(c, cols, nc, W.Ra, nc, false, T[k + 1], cols, spare, cols, st, &fl);
    launch_copy2d(c, cols, spare, cols, T[k + 1], cols, 1.0, 0.0, st);
    tr[k + 1] = c;
  }

  void qr_pass() {
    for (int k = 0; k < K - 1; ++k) {
      qr_step(X, xr, k, xspare);
      qr_step(Z, zr, k, zspare);
      update_envs(k);
    }
    peak_rank = std::max(peak_rank, *std::max_element(xr.begin(), xr.end()));
  }

  // Returns the local residual res_k before the solve.
  double solve_core(int k) {
    const int p = xr[k], t = xr[k + 1];
    const int N = p * n[k] * t;
    local_rhs(p, n[k], sb(k), sb(k + 1), t, Eb[k], B(k), Eb[k + 1], W.Tb, W.g, st, &fl);
    tb_k = k;
    if (with_u)  // g -= (projected) A u, in FP64
      apply_sub(k, p, ur[k], ur[k + 1], t, EuA[k], U[k], EuA[k + 1], W.g, W.ye);
    const Plan& pl = plan(k);
    launch_local_block_inv(p, n[k], t, R(k), R(k + 1), EA[k], EA[k + 1], pl.bk_beg, pl.bk_b, pl.bk_e, pl.bk_v,
                           W.binv, st);
    // the CG's fused apply (x = z); for sparse plans the initial A x is the same apply on
    // X[k], whose split partials the CG init sums itself
    FusedArgs f;
    const bool fused = !pl.dense;
    if (fused) {
      f.L = EA[k];
      f.x = W.z;
      f.Rt = EA[k + 1];
      f.partial = W.fpart;
      f.p = p;
      f.q = p;
      f.s = t;
      f.t = t;
      f.Rl = R(k);
      f.Rr = R(k + 1);
      f.n = n[k];
      set_terms(f, pl);
      f.stage = W.stage;
      f.stage_bytes = W.stage_bytes;
      f.ksplit = fused_apply_splits(f, pl.sp_ap_max, W.fpart_cap);
      FusedArgs f0 = f;
      f0.x = X[k];
      const double flops0 = 2.0 * p * p * t * pl.sp_nslot + 2.0 * p * t * t * pl.sp_n_ap;
      launch_fused_apply(f0, flops0, st, 0);
      fl.total += flops0;
    } else {
      apply(k, p, p, t, t, EA[k], X[k], EA[k + 1], W.q, nullptr);
    }
    applies++;
    CgIterArgs a;
    a.N = N;
    a.x = X[k];
    a.r = W.r;
    a.z = W.z;
    a.p = W.p;
    a.q = W.w;
    a.scal = W.scal;
    a.flag = W.flag;
    a.parts = W.part;
    a.maxit = o.cg_maxit;
    a.n = n[k];
    a.t = t;
    a.nb_upd = cg_dir_blocks(N);
    a.nb_dir = cg_dir_blocks(N);
    set_block_precond(a, n[k], t, W.binv);
    if (fused) {
      a.ksplit = f.ksplit;
      a.partial = W.fpart;
      a.tiles_n = (t + 31) / 32;
      a.ntiles = ((p + 31) / 32) * a.tiles_n;
    }
    launch_cg_init2(a, W.g, fused ? nullptr : W.q, o.tol, st);
    auto readback = [&]() {
      hip_check(hipMemcpyAsync(W.host_pinned, W.flag, (CG_RES_COPY + 2) * sizeof(int), hipMemcpyDeviceToHost, st),
                "flag readback");
      sync();
    };
    // FP64: no readback before the first chunk (its kernels return at once when the
    // initial residual already meets the target); low precision needs the initial
    // residual to steer the refinement
    const bool early = o.precision == 0 || pl.dense;
    double res = 0.0;
    int done = 0;
    if (!early) {
      readback();
      res = *reinterpret_cast<volatile double*>(static_cast<char*>(W.host_pinned) + CG_RES_COPY * sizeof(int));
      if (!std::isfinite(res)) nan_seen = 1;
      done = hint()[0];
    }
    // fused evaluation from the nonzero lists for sparse plans
    const size_t m_need = (size_t)pl.Rl * n[k] * n[k] * (size_t)t * t;
    const bool explicit_mat = pl.dense && !done && (size_t)N <= W.bloc_n && m_need <= W.mloc_cap;
    if (explicit_mat) {
      launch_local_matrix(p, n[k], t, pl.Rl, pl.Rr, EA[k], pl.A2, EA[k + 1], W.Mloc, W.Bloc, st);
      fl.total += 2.0 * m_need * pl.Rr + 2.0 * (double)N * N * pl.Rl;
    }
    if (fused) {
      f.skip = W.flag + CG_DONE;
      // the apply also forms the partials of (z, B z): one CG kernel per iteration
      const int nd = fused_dot_count(f);
      if (nd <= CG_DOT_MAX) {
        f.dots = W.part + CG_DOT_OFFSET;
        a.ndots = nd;
        cg_step_shape(a);
      }
    } else {
      a.ksplit = 0;
      a.w = W.q;
    }
    const double apply_flops = 2.0 * p * p * t * pl.sp_nslot + 2.0 * p * t * t * pl.sp_n_ap;
    // precision > 0: inner CG with low-precision applies, restarted on the residual
    // recomputed in FP64 until that residual meets the target (local refinement).
    // The best FP64-checked iterate is kept; a restart that does not lower the FP64
    // residual (the low-precision operator is too far from the FP64 one for this
    // local system) returns to that iterate and finishes the solve in FP64.
    int prec = fused ? o.precision : 0;
    const int lp_pass_cap = 100;
    const int chunk = 8;
    int total_its = 0;
    const bool converged_at_entry = done;
    double res_best = res;
    double* xbest = W.ye;
    if (prec && !converged_at_entry) launch_copy2d(1, N, X[k], N, xbest, N, 1.0, 0.0, st);
    auto fp64_restart = [&]() {
      apply(k, p, p, t, t, EA[k], X[k], EA[k + 1], W.q, nullptr);
      applies++;
      a.keep_thr = 1;
      a.maxit = o.cg_maxit - total_its;
      launch_cg_init2(a, W.g, W.q, o.tol, st);
      a.keep_thr = 0;
      readback();
      done = hint()[0];
      return *reinterpret_cast<volatile double*>(static_cast<char*>(W.host_pinned) + CG_RES_COPY * sizeof(int));
    };
    for (int refine = 0;; ++refine) {
      int kit = 0;
      const int budget = prec ? std::min(o.cg_maxit - total_its, lp_pass_cap) : o.cg_maxit - total_its;
      a.maxit = budget;
      const size_t pmark = profile_mark();
      const double fl0 = fl.total, fll0 = fl_low;
      // the first chunk covers as many iterations as this core's previous local solve
      // took, so that one status readback usually suffices; later chunks are short
      const int phys = orient ? K - 1 - k : k;
      const int first = refine == 0 ? std::min(48, std::max(chunk, cg_last[phys] + 1)) : chunk;
      while (!done && kit <= budget) {
        const int cn = kit == 0 ? first : chunk;
        for (int c = 0; c < cn && kit <= budget; ++c, ++kit) {
          set_profile_tag(kit);
          if (fused) {
            launch_fused_apply(f, apply_flops, st, prec);
            fl.total += apply_flops;
            if (prec) fl_low += apply_flops;
          } else if (explicit_mat) {
            launch_dense_matvec(N, W.Bloc, W.z, W.q, W.flag + CG_DONE, st);
            fl.total += 2.0 * (double)N * N;
          } else {
            apply(k, p, p, t, t, EA[k], W.z, EA[k + 1], W.q, W.flag + CG_DONE);
          }
          if (a.ndots > 0) {
            launch_cg_step(a, kit, st);
          } else {
            launch_cg_reduce_dir(a, kit, st);
            launch_cg_update2(a, kit, st);
          }
        }
        readback();
        done = hint()[0];
      }
      set_profile_tag(-1);
      bool entry_done = false;
      if (early && refine == 0) {
        // the initial residual, read back with the first chunk's status (the init
        // kernel set the stop flag when it already met the target: nothing ran)
        res = *reinterpret_cast<volatile double*>(static_cast<char*>(W.host_pinned) + CG_RES_COPY * sizeof(int));
        if (!std::isfinite(res)) nan_seen = 1;
        entry_done = res <= 0.5 * o.tol || o.cg_maxit <= 0;
      }
      // the apply of launch index k runs before iteration k's convergence test, so a
      // pass that stopped after `its` iterations ran its + 1 applies; later launches
      // of the last chunk returned at once and are not counted
      const int its = hint()[1];
      const int ran = entry_done ? 0 : std::min(kit, its + 1);
      profile_drop_from(pmark, ran);
      if (kit > 0) {
        const double frac = (double)ran / kit;
        fl.total = fl0 + (fl.total - fl0) * frac;
        fl_low = fll0 + (fl_low - fll0) * frac;
      }
      applies += ran;
      total_its += its;
      if (refine == 0) cg_last[phys] = entry_done ? 0 : its;
      if (prec == 0 || converged_at_entry || total_its >= o.cg_maxit) break;
      const double res_now = fp64_restart();
      refinements++;
      if (done) break;
      // under the outer refinement a low-precision pass that lowered the FP64 residual is
      // kept as it stands (the outer loop carries the correction); one that did not falls
      // back below
      if (ir_inner && std::isfinite(res_now) && res_now < res_best) break;
      if (std::isfinite(res_now) && res_now < 0.9 * res_best && refine < 30) {
        res_best = res_now;
        launch_copy2d(1, N, X[k], N, xbest, N, 1.0, 0.0, st);
        continue;
      }
      if (!(std::isfinite(res_now) && res_now < res_best)) {
        launch_copy2d(1, N, xbest, N, X[k], N, 1.0, 0.0, st);
        fp64_restart();
        if (done) break;
      }
      prec = 0;
      fallbacks++;
    }
    cg_iters += total_its;
    if (verbose >= 2)
      fprintf(stderr, "[tnfem]   core %d (orient %d) p %d n %d t %d N %d %s R %d/%d res %.3e cg %d\n", k, orient, p,
              n[k], t, N, pl.dense ? "dense" : "sparse", R(k), R(k + 1), res, total_its);
    return res;
  }

  // Truncation and enrichment of core k, in four phases so that a lockstep batch can
  // issue the QR / SVD of all its requests as shared launches between them:
  //   trunc_begin  -> QR job of the unfolding, SVD job of its R factor
  //   trunc_rank   -> U, V^T, truncation rank (read back; the caller synchronises)
  //   enrich_begin -> truncated core, residual projections; QR jobs of the new Z
  //                   core and of the enriched basis [U | residual]
  //   enrich_end   -> carry Q^T x into core k + 1, ranks, interface updates
  struct TruncState {
    int p = 0, nk = 0, t = 0, M = 0, Nn = 0, c = 0, rk = 0, rnew = 0, cz = 0;
    bool tall = true;
    QrJob qr, zqr, aqr;
    SvdJob svd;
  };

  void trunc_begin(int k, TruncState& s) {
    s.p = xr[k];
    s.nk = n[k];
    s.t = xr[k + 1];
    s.M = s.p * s.nk;
    s.Nn = s.t;
    s.c = std::min(s.M, s.Nn);
    s.tall = s.M >= s.Nn;
    const int M = s.M, Nn = s.Nn;
    // Only the left singular vectors of x and S are needed (the truncated x is the
    // projection U_rk U_rk^T x), so the Jacobi SVD runs on the matrix whose normalised
    // columns are those vectors and accumulates no rotations.
    if (s.tall) {
      // x = Q R, R = U_R S V^T: Jacobi on R, U_R from its columns; U = Q U_R
      s.qr = QrJob{M, Nn, Nn, Nn, Nn, X[k], W.Qx, W.Rx, W.qrws, W.qrws_cap};
      s.svd = SvdJob{Nn, Nn, W.Rx, W.UR, W.S, W.V, W.qrws, 0, true};
    } else {
      // x^T = Q R  =>  x = R^T Q^T: Jacobi on R^T, whose columns give U directly
      launch_core_transpose(M, 1, Nn, X[k], W.xT, st);
      s.qr = QrJob{Nn, M, M, M, M, W.xT, W.Qx, W.Rx, W.qrws, W.qrws_cap};
      s.svd = SvdJob{M, M, W.Rx, W.UR, W.S, W.V, W.qrws, 1, true};
    }
  }

  void trunc_rank(int k, TruncState& s) {
    (void)k;
    const int M = s.M, Nn = s.Nn, c = s.c;
    if (s.tall) {
      gemm_plain(M, Nn, Nn, W.Qx, Nn, false, W.UR, Nn, W.Ur, c, st, &fl);
    } else {
      launch_copy2d(M, M, W.UR, M, W.Ur, c, 1.0, 0.0, st);
    }
    const double trtol = o.tol / std::sqrt((double)std::max(K - 1, 1));
    launch_trunc_rank(c, W.S, trtol, o.rank_cap, W.drank, st);
    hip_check(hipMemcpyAsync(W.host_pinned, W.drank, sizeof(int), hipMemcpyDeviceToHost, st), "rank readback");
  }

  void enrich_begin(int k, TruncState& s) {
    const int p = s.p, nk = s.nk, t = s.t, M = s.M, Nn = s.Nn, c = s.c;
    const int rk = hint()[0];
    s.rk = rk;
    const int pz = zr[k], tz = zr[k + 1];
    // enrichment: residual on (left X, right Z) interfaces, as many columns as the cap
    // leaves room for
    const int rho_eff = std::max(0, std::min(tz, std::min(o.rank_cap - rk, M - rk)));
    const int rnew = rk + rho_eff;
    s.rnew = rnew;
    // xt = U_rk (U_rk^T x) (U_rk: the first rk columns of U, leading dimension c), which
    // equals U_rk diag(S_rk) V^T_rk; beside it the first products of the two loads
    GemmSet g;
    g.add(plain_desc(rk, Nn, M, W.Ur, c, true, X[k], Nn, W.SVt, Nn));
    g.add(rhs1_desc(pz, nk, sb(k), sb(k + 1), Ezb[k], B(k), W.Tbz));
    if (rho_eff > 0 && tb_k != k) g.add(rhs1_desc(p, nk, sb(k), sb(k + 1), Eb[k], B(k), W.Tb));
    g.launch(st, &fl);
    tbz_k = k;
    if (rho_eff > 0) tb_k = k;
    g.add(plain_desc(M, Nn, rk, W.Ur, c, false, W.SVt, Nn, W.xt, Nn));
    g.add(rhs2_desc(pz, nk, sb(k + 1), tz, W.Tbz, Ezb[k + 1], W.gz));
    if (rho_eff > 0) g.add(rhs2_desc(p, nk, sb(k + 1), tz, W.Tb, Ezb[k + 1], W.ge));
    g.launch(st, &fl);
    const int mz = pz * nk;
    s.cz = std::min(mz, tz);
    s.zqr = QrJob{mz, tz, tz, s.cz, tz, W.gz, Z[k], W.Rz, W.qrwsz, W.qrwsz_cap};
    if (rho_eff > 0 && !plan(k).dense && !with_u) {
      // both residuals (on the Z interfaces -> new Z_k; on (left X, right Z) -> the
      // enrichment) from their applies, partials in the two halves of the split buffer,
      // subtracted in one launch
      const Plan& pl = plan(k);
      const size_t half = W.fpart_cap / 2;
      const FusedArgs fz = fused_args(k, pz, p, t, tz, EzA[k], W.xt, EzA[k + 1], W.fpart, half);
      const FusedArgs fe = fused_args(k, p, p, t, tz, EA[k], W.xt, EzA[k + 1], W.fpart + half, half);
      const double flz = 2.0 * pz * p * t * pl.sp_nslot + 2.0 * pz * t * tz * pl.sp_n_ap;
      const double fle = 2.0 * p * p * t * pl.sp_nslot + 2.0 * p * t * tz * pl.sp_n_ap;
      launch_fused_apply(fz, flz, st, 0);
      launch_fused_apply(fe, fle, st, 0);
      launch_fused_sum2(fz, W.gz, W.gz, fe, W.ge, W.ge, st);
      fl.total += flz + fle;
    } else {
      // residual projected on the Z interfaces -> new Z_k (QR job)
      apply_sub(k, pz, p, t, tz, EzA[k], W.xt, EzA[k + 1], W.gz, W.yz);
      if (with_u) apply_sub(k, pz, ur[k], ur[k + 1], tz, EzuA[k], U[k], EzuA[k + 1], W.gz, W.yz);
      if (rho_eff > 0) {
        apply_sub(k, p, p, t, tz, EA[k], W.xt, EzA[k + 1], W.ge, W.ye);
        if (with_u) apply_sub(k, p, ur[k], ur[k + 1], tz, EuA[k], U[k], EzuA[k + 1], W.ge, W.ye);
      }
    }
    if (rho_eff == 0) {
      // no room: U_rk (orthonormal columns) is the new core as it stands
      launch_copy2d(M, rk, W.Ur, c, X[k], rk, 1.0, 0.0, st);
      s.aqr = QrJob{};
      return;
    }
    // the augmented basis [U_rk | residual columns]
    launch_copy_concat(M, rk, W.Ur, c, rho_eff, W.ge, tz, W.aug, rnew, st);
    s.aqr = QrJob{M, rnew, rnew, rnew, rnew, W.aug, X[k], W.Ra, W.qrws, W.qrws_cap};
  }

  // the QR jobs of enrich_begin (the enrichment QR only when columns were added)
  static void push_enrich_jobs(const TruncState& s, std::vector<QrJob>& jobs) {
    jobs.push_back(s.zqr);
    if (s.aqr.m > 0) jobs.push_back(s.aqr);
  }

  void enrich_end(int k, TruncState& s) {
    const int M = s.M, Nn = s.Nn, rnew = s.rnew;
    // W = Q^T xt (rnew x Nn); X_{k+1} <- W X_{k+1}, issued with the interface updates
    const int cols = n[k + 1] * xr[k + 2];
    const GemmDesc wm = plain_desc(rnew, Nn, M, X[k], rnew, true, W.xt, Nn, W.Wm, Nn);
    const GemmDesc carry = plain_desc(rnew, cols, Nn, W.Wm, Nn, false, X[k + 1], cols, xspare, cols);
    xr[k + 1] = rnew;
    peak_rank = std::max(peak_rank, rnew);
    zr[k + 1] = s.cz;
    update_envs(k, &wm, &carry);
    std::swap(X[k + 1], xspare);
  }

  void truncate_enrich(int k) {
    TruncState s;
    trunc_begin(k, s);
    launch_qr(s.qr.m, s.qr.n, s.qr.A, s.qr.lda, s.qr.Q, s.qr.ldq, s.qr.R, s.qr.ldr, s.qr.ws, s.qr.ws_cap, st);
    launch_jacobi_svd(s.svd.n, s.svd.G, s.svd.ldg, s.svd.U, s.svd.S, s.svd.V, s.svd.ws, st, s.svd.trans,
                      s.svd.left_only);
    trunc_rank(k, s);
    sync();
    enrich_begin(k, s);
    std::vector<QrJob> jobs;
    push_enrich_jobs(s, jobs);
    launch_qr_batch(jobs, st);  // independent: one launch, one workgroup each
    enrich_end(k, s);
  }

  // ---- outer refinement (forward orientation throughout)

  // The current iterate becomes u; the sweep restarts from random cores on the correction
  // equation A d = b - A u (orthogonalisation and right interfaces rebuilt, those of u too).
  void begin_correction(IrBuffers& B, uint64_t seed_x, uint64_t seed_z) {
    tb_k = tbz_k = -1;
    if (!with_u) {
      U = B.U;
      uspare = B.uspare;
      EuA = B.EuA;
      EzuA = B.EzuA;
      with_u = true;
      ur = xr;
      for (int k = 0; k < K; ++k)
        hip_check(hipMemcpyAsync(U[k], X[k], (size_t)xr[k] * n[k] * xr[k + 1] * 8, hipMemcpyDeviceToDevice, st),
                  "copy u");
    }
    upload_initial(seed_x, seed_z);
    reverse();
    qr_pass();
    reverse();
  }

  // Reads back the truncation rank written to W.drank.
  int read_rank() {
    hip_check(hipMemcpyAsync(W.host_pinned, W.drank, sizeof(int), hipMemcpyDeviceToHost, st), "rank readback");
    sync();
    return hint()[0];
  }

  // u <- round(u + d) with d the current iterate X: the block sum of the two TTs,
  // right-to-left orthogonalisation (QR of each transposed unfolding), then left-to-right
  // SVD truncation at rtol (relative to the whole TT) with ranks at most cap.
  // Returns ||d|| / ||u + d|| (FP64 norms: d's on the host, the sum's from its first core).
  double add_correction(IrBuffers& B, double rtol, int cap) {
    // ||d|| on the host (d's cores are a few hundred KB)
    std::vector<std::vector<double>> dc(K);
    for (int k = 0; k < K; ++k) {
      dc[k].resize((size_t)xr[k] * n[k] * xr[k + 1]);
      hip_check(hipMemcpyAsync(dc[k].data(), X[k], dc[k].size() * 8, hipMemcpyDeviceToHost, st), "download d");
    }
    sync();
    const double dnorm = hostla::tt_norm(n, xr, dc);
    std::vector<int> sr(K + 1);
    sr[0] = 1;
    sr[K] = 1;
    for (int k = 1; k < K; ++k) sr[k] = ur[k] + xr[k];
    for (int k = 0; k < K; ++k) {
      const int rl = sr[k], rr = sr[k + 1];
      hip_check(hipMemsetAsync(B.Sum[k], 0, (size_t)rl * n[k] * rr * 8, st), "clear sum core");
      const int roff = k == 0 ? 0 : ur[k], coff = k == K - 1 ? 0 : ur[k + 1];
      launch_copy2d(ur[k] * n[k], ur[k + 1], U[k], ur[k + 1], B.Sum[k], rr, 1.0, 0.0, st);
      launch_copy2d(xr[k] * n[k], xr[k + 1], X[k], xr[k + 1], B.Sum[k] + (size_t)roff * n[k] * rr + coff, rr, 1.0,
                    1.0, st);
    }
    // right-to-left: core k = R^T Q^T with Q^T row-orthonormal; R^T goes into core k - 1
    for (int k = K - 1; k > 0; --k) {
      const int rl = sr[k], rr = sr[k + 1], nk = n[k];
      const int m = rr * nk, c = std::min(m, rl);
      launch_core_transpose(rl, nk, rr, B.Sum[k], B.t1, st);  // [rr][n][rl]: (rr n) x rl
      launch_qr(m, rl, B.t1, rl, B.t2, c, B.svt, rl, B.svdws, B.svdws_cap, st);
      launch_core_transpose(rr, nk, c, B.t2, B.Sum[k], st);   // [c][n][rr]
      launch_core_transpose(c, 1, rl, B.svt, B.t1, st);  // R^T: rl x c
      const int pm = sr[k - 1] * n[k - 1];
      gemm_plain(pm, c, rl, B.Sum[k - 1], rl, false, B.t1, c, B.t2, c, st, &fl);
      launch_copy2d(pm, c, B.t2, c, B.Sum[k - 1], c, 1.0, 0.0, st);
      sr[k] = c;
    }
    // ||u + d|| = ||core 0|| now
    std::vector<double> c0((size_t)sr[0] * n[0] * sr[1]);
    hip_check(hipMemcpyAsync(c0.data(), B.Sum[0], c0.size() * 8, hipMemcpyDeviceToHost, st), "download core 0");
    sync();
    double snorm = 0.0;
    for (double v : c0) snorm += v * v;
    snorm = std::sqrt(snorm);
    // left-to-right SVD truncation
    const double ktol = rtol / std::sqrt((double)std::max(K - 1, 1));
    for (int k = 0; k < K - 1; ++k) {
      const int M = sr[k] * n[k], Nn = sr[k + 1], c = std::min(M, Nn);
      svd_device(M, Nn, B.Sum[k], B.su, B.ss, B.svt, B.svdws, B.svdws_cap, st);
      launch_trunc_rank(c, B.ss, ktol, cap, W.drank, st);
      const int rk = read_rank();
      launch_copy2d(M, rk, B.su, c, B.Sum[k], rk, 1.0, 0.0, st);
      launch_scale_rows(rk, Nn, B.ss, B.svt, Nn, B.t2, st);  // diag(S) V^T, rk x Nn
      const int cols = n[k + 1] * sr[k + 2];
      gemm_plain(rk, cols, Nn, B.t2, Nn, false, B.Sum[k + 1], cols, B.t1, cols, st, &fl);
      launch_copy2d(rk, cols, B.t1, cols, B.Sum[k + 1], cols, 1.0, 0.0, st);
      sr[k + 1] = rk;
    }
    for (int k = 0; k < K; ++k)
      hip_check(hipMemcpyAsync(U[k], B.Sum[k], (size_t)sr[k] * n[k] * sr[k + 1] * 8, hipMemcpyDeviceToDevice, st),
                "store u");
    ur = sr;
    peak_rank = std::max(peak_rank, *std::max_element(sr.begin(), sr.end()));
    return snorm > 0.0 ? dnorm / snorm : dnorm;
  }

  // The refined u becomes the iterate (for the download of the result).
  void take_u() {
    for (int k = 0; k < K; ++k)
      hip_check(hipMemcpyAsync(X[k], U[k], (size_t)ur[k] * n[k] * ur[k + 1] * 8, hipMemcpyDeviceToDevice, st),
                "copy u");
    xr = ur;
  }

  double half_sweep() {
    double mr = 0.0;
    for (int k = 0; k < K; ++k) {
      const double res = solve_core(k);
      mr = std::max(mr, res);
      if (nan_seen) return NAN;
      if (k < K - 1) truncate_enrich(k);
    }
    return mr;
  }
};

}  // namespace

// ----------------------------------------------------------------------------- lockstep batches

namespace {

// Device + pinned host copies of the per-request argument arrays of the shared launches.
struct BatchArgs {
  FusedArgs* d_f = nullptr;
  CgIterArgs* d_a = nullptr;
  FusedArgs* h_f = nullptr;
  CgIterArgs* h_a = nullptr;
  const DeviceAllocator& alloc;
  BatchArgs(int n, const DeviceAllocator& a) : alloc(a) {
    d_f = static_cast<FusedArgs*>(alloc.allocate(sizeof(FusedArgs) * n));
    d_a = static_cast<CgIterArgs*>(alloc.allocate(sizeof(CgIterArgs) * n));
    hip_check(hipHostMalloc(reinterpret_cast<void**>(&h_f), sizeof(FusedArgs) * n, hipHostMallocDefault),
              "hipHostMalloc batch args");
    hip_check(hipHostMalloc(reinterpret_cast<void**>(&h_a), sizeof(CgIterArgs) * n, hipHostMallocDefault),
              "hipHostMalloc batch args");
  }
  ~BatchArgs() {
    alloc.release(d_f);
    alloc.release(d_a);
    if (h_f) (void)hipHostFree(h_f);
    if (h_a) (void)hipHostFree(h_a);
  }
};

// The local solves of core k of several sweeps (same chain, same orientation, same
// options): per request exactly the steps of Sweep::solve_core, with the CG iterations
// of all requests issued as shared launches (one fused apply per rank class and
// operand precision, one direction update, one vector update per iteration).  Returns
// each request's local residual.
std::vector<double> batch_solve_core(std::vector<Sweep*>& S, int k, BatchArgs& args, hipStream_t st) {
  const int nb = (int)S.size();
  struct Loc {
    int p = 0, t = 0, N = 0;
    const Plan* pl = nullptr;
    CgIterArgs a;
    FusedArgs f;
    bool fused = false, explicit_mat = false, done = false;
    double res = 0.0, apply_flops = 0.0, fl0 = 0.0;
  };
  std::vector<Loc> L(nb);
  for (int r = 0; r < nb; ++r) {
    Sweep& w = *S[r];
    Workspace& W = w.W;
    Loc& c = L[r];
    set_gemm_splitk_buffer(W.splitk, W.splitk_cap);
    c.p = w.xr[k];
    c.t = w.xr[k + 1];
    c.N = c.p * w.n[k] * c.t;
    c.pl = &w.plan(k);
    local_rhs(c.p, w.n[k], w.sb(k), w.sb(k + 1), c.t, w.Eb[k], w.B(k), w.Eb[k + 1], W.Tb, W.g, st, &w.fl);
    w.tb_k = k;
    launch_local_block_inv(c.p, w.n[k], c.t, w.R(k), w.R(k + 1), w.EA[k], w.EA[k + 1], c.pl->bk_beg, c.pl->bk_b,
                           c.pl->bk_e, c.pl->bk_v, W.binv, st);
    w.apply(k, c.p, c.p, c.t, c.t, w.EA[k], w.X[k], w.EA[k + 1], W.q, nullptr);
    w.applies++;
    CgIterArgs& a = c.a;
    a.N = c.N;
    a.x = w.X[k];
    a.r = W.r;
    a.z = W.z;
    a.p = W.p;
    a.q = W.w;
    a.scal = W.scal;
    a.flag = W.flag;
    a.parts = W.part;
    a.maxit = w.o.cg_maxit;
    a.n = w.n[k];
    a.t = c.t;
    a.nb_upd = cg_dir_blocks(c.N);
    a.nb_dir = cg_dir_blocks(c.N);
    set_block_precond(a, w.n[k], c.t, W.binv);
    launch_cg_init2(a, W.g, W.q, w.o.tol, st);
    hip_check(hipMemcpyAsync(W.host_pinned, W.flag, (CG_RES_COPY + 2) * sizeof(int), hipMemcpyDeviceToHost, st),
              "flag readback");
  }
  hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
  int max_n = 0;
  for (int r = 0; r < nb; ++r) {
    Sweep& w = *S[r];
    Workspace& W = w.W;
    Loc& c = L[r];
    const Plan& pl = *c.pl;
    c.res = *reinterpret_cast<volatile double*>(static_cast<char*>(W.host_pinned) + CG_RES_COPY * sizeof(int));
    if (!std::isfinite(c.res)) w.nan_seen = 1;
    c.done = w.hint()[0] != 0;
    c.fused = !pl.dense;
    const size_t m_need = (size_t)pl.Rl * w.n[k] * w.n[k] * (size_t)c.t * c.t;
    c.explicit_mat = pl.dense && !c.done && (size_t)c.N <= W.bloc_n && m_need <= W.mloc_cap;
    if (c.explicit_mat) {
      launch_local_matrix(c.p, w.n[k], c.t, pl.Rl, pl.Rr, w.EA[k], pl.A2, w.EA[k + 1], W.Mloc, W.Bloc, st);
      w.fl.total += 2.0 * m_need * pl.Rr + 2.0 * (double)c.N * c.N * pl.Rl;
    }
    FusedArgs& f = c.f;
    if (c.fused) {
      f.L = w.EA[k];
      f.x = W.z;
      f.Rt = w.EA[k + 1];
      f.partial = W.fpart;
      f.p = c.p;
      f.q = c.p;
      f.s = c.t;
      f.t = c.t;
      f.Rl = w.R(k);
      f.Rr = w.R(k + 1);
      f.n = w.n[k];
      set_terms(f, pl);
      f.stage = W.stage;
      f.stage_bytes = W.stage_bytes;
      f.ksplit = fused_apply_splits(f, pl.sp_ap_max, W.fpart_cap);
      f.skip = W.flag + CG_DONE;
      fused_prepare(f);
      c.a.ksplit = f.ksplit;
      c.a.partial = W.fpart;
      c.a.tiles_n = (c.t + 31) / 32;
      c.a.ntiles = ((c.p + 31) / 32) * c.a.tiles_n;
      const int nd = fused_dot_count(f);
      if (nd <= CG_DOT_MAX) {
        f.dots = W.part + CG_DOT_OFFSET;
        c.a.ndots = nd;
        cg_step_shape(c.a);
      }
    } else {
      c.a.ksplit = 0;
      c.a.w = W.q;
    }
    c.apply_flops = 2.0 * c.p * c.p * c.t * pl.sp_nslot + 2.0 * c.p * c.t * c.t * pl.sp_n_ap;
    c.fl0 = w.fl.total;
    max_n = std::max(max_n, w.n[k]);
  }
  // The local refinement of Sweep::solve_core, request by request: passes of CG
  // iterations (low precision: at most 100 iterations each) issued in lockstep for all
  // requests still iterating, then, for the requests whose low-precision pass ended, the
  // FP64 restart and the same decisions as the single solve (continue in low precision,
  // go back to the best FP64-checked iterate, finish in FP64).
  const int maxit = S[0]->o.cg_maxit;
  const int lp_pass_cap = 100;
  struct Pass {
    int prec = 0, refine = 0, total_its = 0, applies = 0;
    bool conv_entry = false, finished = false;
    double res_best = 0.0;
  };
  std::vector<Pass> ps(nb);
  for (int r = 0; r < nb; ++r) {
    Sweep& w = *S[r];
    Pass& q = ps[r];
    q.prec = L[r].fused ? w.o.precision : 0;
    q.conv_entry = q.finished = L[r].done;
    q.res_best = L[r].res;
    if (q.prec && !q.conv_entry) launch_copy2d(1, L[r].N, w.X[k], L[r].N, w.W.ye, L[r].N, 1.0, 0.0, st);
  }
  // FP64 restart of request r: the residual of its iterate recomputed in FP64, the CG
  // restarted from it with the kept threshold (read back by the caller)
  auto restart = [&](int r) {
    Sweep& w = *S[r];
    Loc& c = L[r];
    set_gemm_splitk_buffer(w.W.splitk, w.W.splitk_cap);
    w.apply(k, c.p, c.p, c.t, c.t, w.EA[k], w.X[k], w.EA[k + 1], w.W.q, nullptr);
    w.applies++;
    c.a.keep_thr = 1;
    c.a.maxit = maxit - ps[r].total_its;
    launch_cg_init2(c.a, w.W.g, w.W.q, w.o.tol, st);
    c.a.keep_thr = 0;
    hip_check(hipMemcpyAsync(w.W.host_pinned, w.W.flag, (CG_RES_COPY + 2) * sizeof(int), hipMemcpyDeviceToHost, st),
              "flag readback");
  };
  for (;;) {
    // requests in a pass, split by apply kind and operand precision
    std::vector<int> cg, other, tiled, bykind[2][3];
    for (int r = 0; r < nb; ++r) {
      if (ps[r].finished) continue;
      cg.push_back(r);
      if (!L[r].fused) other.push_back(r);
      else if (fused_kind(L[r].f) == FUSED_TILED) tiled.push_back(r);
      else bykind[fused_kind(L[r].f)][ps[r].prec].push_back(r);
      L[r].a.maxit = ps[r].prec ? std::min(maxit - ps[r].total_its, lp_pass_cap) : maxit - ps[r].total_its;
    }
    if (cg.empty()) break;
    int kit = 0, bmax = 0;
    for (int r : cg) bmax = std::max(bmax, L[r].a.maxit);
    std::vector<double> fl0(nb), fll0(nb);
    for (int r : cg) {
      fl0[r] = S[r]->fl.total;
      fll0[r] = S[r]->fl_low;
    }
    FusedBatch fb[2][3];  // shared launches of the one-pass kernels; ranks above 64 per request
    int nf = 0;
    for (int kd = 0; kd < 2; ++kd)
      for (int pr = 0; pr < 3; ++pr) {
        FusedBatch& b = fb[kd][pr];
        const std::vector<int>& ids = bykind[kd][pr];
        b.args = args.d_f + nf;
        b.nreq = (int)ids.size();
        b.zoff[0] = 0;
        for (int i = 0; i < b.nreq; ++i) {
          const FusedArgs& f = L[ids[i]].f;
          args.h_f[nf + i] = f;
          b.zoff[i + 1] = b.zoff[i] + f.ksplit;
          b.bpw = std::max(b.bpw, fused16_bpw(f));
        }
        nf += b.nreq;
      }
    // requests whose apply forms (z, B z) take one step kernel per iteration, the others
    // the direction and update kernels; the argument array holds the step group first
    // (step requests grouped by their block size: 64-thread blocks first)
    std::vector<int> order;
    for (int r : cg)
      if (L[r].a.ndots > 0 && L[r].a.nt_step == 64) order.push_back(r);
    const int nstep64 = (int)order.size();
    for (int r : cg)
      if (L[r].a.ndots > 0 && L[r].a.nt_step != 64) order.push_back(r);
    const int nstep = (int)order.size();
    for (int r : cg)
      if (L[r].a.ndots == 0) order.push_back(r);
    CgBatch step[2], dir, upd;
    step[0].args = args.d_a;
    step[0].nreq = nstep64;
    step[0].nt = 64;
    step[1].args = args.d_a + nstep64;
    step[1].nreq = nstep - nstep64;
    step[1].nt = 256;
    dir.args = upd.args = args.d_a + nstep;
    dir.nreq = upd.nreq = (int)cg.size() - nstep;
    for (int i = 0; i < (int)order.size(); ++i) args.h_a[i] = L[order[i]].a;
    for (int i = 0; i < nstep; ++i) {
      const CgIterArgs& a = L[order[i]].a;
      cg_step_check(a);
      CgBatch& sb = step[i < nstep64 ? 0 : 1];
      const int j = i < nstep64 ? i : i - nstep64;
      sb.boff[j + 1] = sb.boff[j] + a.nb_step;
    }
    for (int i = 0; i < dir.nreq; ++i) {
      const CgIterArgs& a = L[order[nstep + i]].a;
      dir.boff[i + 1] = dir.boff[i] + a.nb_dir;
      upd.boff[i + 1] = upd.boff[i] + a.nb_upd;
    }
    if (nf)
      hip_check(hipMemcpyAsync(args.d_f, args.h_f, sizeof(FusedArgs) * nf, hipMemcpyHostToDevice, st),
                "batch args upload");
    hip_check(hipMemcpyAsync(args.d_a, args.h_a, sizeof(CgIterArgs) * cg.size(), hipMemcpyHostToDevice, st),
              "batch args upload");
    const int chunk = 8;
    bool any = true;
    while (any && kit <= bmax) {
      for (int c = 0; c < chunk && kit <= bmax; ++c, ++kit) {
        for (int kd = 0; kd < 2; ++kd)
          for (int pr = 0; pr < 3; ++pr)
            if (fb[kd][pr].nreq) launch_fused_apply_batch(fb[kd][pr], max_n, kd, st, pr);
        for (int r : tiled) launch_fused_apply(L[r].f, 0.0, st, ps[r].prec);
        for (int r : cg) {
          if (!L[r].fused) continue;
          S[r]->fl.total += L[r].apply_flops;
          if (ps[r].prec) S[r]->fl_low += L[r].apply_flops;
        }
        for (int r : other) {
          Sweep& w = *S[r];
          if (L[r].explicit_mat) {
            launch_dense_matvec(L[r].N, w.W.Bloc, w.W.z, w.W.q, w.W.flag + CG_DONE, st);
            w.fl.total += 2.0 * (double)L[r].N * L[r].N;
          } else {
            set_gemm_splitk_buffer(w.W.splitk, w.W.splitk_cap);
            w.apply(k, L[r].p, L[r].p, L[r].t, L[r].t, w.EA[k], w.W.z, w.EA[k + 1], w.W.q, w.W.flag + CG_DONE);
          }
        }
        launch_cg_step_batch(step[0], kit, st);
        launch_cg_step_batch(step[1], kit, st);
        launch_cg_reduce_dir_batch(dir, kit, st);
        launch_cg_update2_batch(upd, kit, st);
      }
      for (int r : cg)
        hip_check(hipMemcpyAsync(S[r]->W.host_pinned, S[r]->W.flag, 2 * sizeof(int), hipMemcpyDeviceToHost, st),
                  "flag readback");
      hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
      any = false;
      for (int r : cg) any = any || S[r]->hint()[0] == 0;
    }
    // the apply of launch index i runs before iteration i's convergence test, so a pass
    // that stopped after `its` iterations ran its + 1 applies
    std::vector<int> rs;
    for (int r : cg) {
      Sweep& w = *S[r];
      Pass& q = ps[r];
      const int its = w.hint()[1];
      const int ran = std::min(kit, its + 1);
      if (kit > 0) {
        const double frac = (double)ran / kit;
        w.fl.total = fl0[r] + (w.fl.total - fl0[r]) * frac;
        w.fl_low = fll0[r] + (w.fl_low - fll0[r]) * frac;
      }
      q.applies += ran;
      q.total_its += its;
      if (q.prec == 0 || q.conv_entry || q.total_its >= maxit) {
        q.finished = true;
        continue;
      }
      rs.push_back(r);
    }
    if (rs.empty()) continue;
    for (int r : rs) restart(r);
    hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
    std::vector<int> back;
    for (int r : rs) {
      Sweep& w = *S[r];
      Pass& q = ps[r];
      const double res_now =
          *reinterpret_cast<volatile double*>(static_cast<char*>(w.W.host_pinned) + CG_RES_COPY * sizeof(int));
      w.refinements++;
      if (w.hint()[0]) {
        q.finished = true;
        continue;
      }
      if (std::isfinite(res_now) && res_now < 0.9 * q.res_best && q.refine < 30) {
        q.res_best = res_now;
        launch_copy2d(1, L[r].N, w.X[k], L[r].N, w.W.ye, L[r].N, 1.0, 0.0, st);
        q.refine++;
        continue;
      }
      if (!(std::isfinite(res_now) && res_now < q.res_best)) {
        launch_copy2d(1, L[r].N, w.W.ye, L[r].N, w.X[k], L[r].N, 1.0, 0.0, st);
        back.push_back(r);
        continue;
      }
      q.prec = 0;
      w.fallbacks++;
      q.refine++;
    }
    if (!back.empty()) {
      for (int r : back) restart(r);
      hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
      for (int r : back) {
        Sweep& w = *S[r];
        Pass& q = ps[r];
        if (w.hint()[0]) {
          q.finished = true;
          continue;
        }
        q.prec = 0;
        w.fallbacks++;
        q.refine++;
      }
    }
  }
  std::vector<double> res(nb);
  for (int r = 0; r < nb; ++r) {
    Sweep& w = *S[r];
    Loc& c = L[r];
    w.applies += ps[r].applies;
    w.cg_iters += ps[r].total_its;
    if (w.verbose >= 2)
      fprintf(stderr, "[tnfem]   core %d (orient %d, batch of %d) p %d n %d t %d N %d %s res %.3e cg %d\n", k,
              w.orient, nb, c.p, w.n[k], c.t, c.N, c.pl->dense ? "dense" : "sparse", c.res, ps[r].total_its);
    res[r] = c.res;
  }
  return res;
}

}  // namespace

static void check_opts(const tnfem_solve_opts& o) {
  TNFEM_REQUIRE(o.rank_cap >= 1 && o.rank_cap <= 252, "rank_cap must be in [1, 252]");
  TNFEM_REQUIRE(o.rho >= 0 && o.rho <= 64, "rho must be in [0, 64]");
  TNFEM_REQUIRE(o.init_rank >= 1 && o.init_rank <= o.rank_cap, "init_rank must be in [1, rank_cap]");
  TNFEM_REQUIRE(o.tol > 0 && std::isfinite(o.tol), "tol must be positive");
  TNFEM_REQUIRE(o.max_sweeps >= 1, "max_sweeps must be >= 1");
  TNFEM_REQUIRE(o.cg_maxit >= 0, "cg_maxit must be >= 0");
  TNFEM_REQUIRE(o.precision >= 0 && o.precision <= 2, "precision must be 0 (FP64), 1 (FP32) or 2 (BF16)");
  TNFEM_REQUIRE(o.ir_max >= 0 && o.ir_sweeps >= 0 && o.ir_tol >= 0 && std::isfinite(o.ir_tol),
                "ir_max, ir_sweeps and ir_tol must be >= 0");
  TNFEM_REQUIRE(o.ir_max == 0 || std::max(o.rank_cap, o.rho) <= 128,
                "outer refinement needs rank_cap <= 128 (the rounding of u + d takes SVDs of 2 rank_cap columns)");
}

static void prepare_workspace(Problem& P, const tnfem_solve_opts& o) {
  const int rho = std::max(o.rho, 1);
  P.ensure_workspace(o.rank_cap, rho);
  if ((size_t)P.ws->cap * P.maxn * (P.ws->cap + rho) * 8 > (size_t)1 << 34)
    fail(TNFEM_EBUDGET, "workspace too large");
}

// Back to the forward orientation, hand the buffer permutation back to the
// workspace and download the solution cores.
static void finish_sweep(Problem& P, Sweep& sw, HostTT& out) {
  if (sw.orient) sw.reverse();
  sw.sync();
  P.ws->X = sw.X;
  P.ws->Z = sw.Z;
  P.ws->Xspare = sw.xspare;
  P.ws->Zspare = sw.zspare;
  P.ws->Xalt = sw.Xalt;
  P.ws->Zalt = sw.Zalt;
  out.modes = sw.n;
  out.ranks = sw.xr;
  out.cores.assign(P.K, {});
  for (int k = 0; k < P.K; ++k) {
    out.cores[k].resize((size_t)sw.xr[k] * sw.n[k] * sw.xr[k + 1]);
    hip_check(hipMemcpyAsync(out.cores[k].data(), sw.X[k], out.cores[k].size() * 8, hipMemcpyDeviceToHost, sw.st),
              "download");
  }
  sw.sync();
}

static void fill_stats(const Sweep& sw, int sweeps, int converged, double last, double seconds,
                       tnfem_solve_stats& stats) {
  stats = tnfem_solve_stats{};
  stats.sweeps = sweeps;
  stats.converged = converged;
  stats.final_max_res = last;
  stats.cg_iters = sw.cg_iters;
  stats.local_applies = sw.applies;
  stats.flops = sw.fl.total;
  stats.seconds = seconds;
  stats.max_rank = *std::max_element(sw.xr.begin(), sw.xr.end());
  stats.peak_rank = std::max(sw.peak_rank, stats.max_rank);
  stats.refinements = sw.refinements;
  stats.low_precision_flops = sw.fl_low;
  stats.precision_fallbacks = sw.fallbacks;
}

int run_solve(Problem& P, const tnfem_solve_opts& o, HostTT& out, tnfem_solve_stats& stats) {
  check_opts(o);
  hip_check(hipSetDevice(P.ctx->device), "hipSetDevice");
  const int rho = std::max(o.rho, 1);
  prepare_workspace(P, o);
  const auto t0 = std::chrono::steady_clock::now();
  tnfem_solve_opts oo = o;
  oo.rho = rho;
  const char* verbose_env = std::getenv("TNFEM_VERBOSE");
  const bool verbose = verbose_env && std::atoi(verbose_env) >= 1;
  if (o.profile) {
    if (!P.ws->profile) P.ws->profile = std::make_unique<GemmProfile>();
    P.ws->profile->reset();
    set_gemm_profile(P.ws->profile.get());
  }
  struct Unset {
    ~Unset() {
      set_gemm_profile(nullptr);
      set_gemm_splitk_buffer(nullptr, 0);
    }
  } unset;
  set_gemm_splitk_buffer(P.ws->splitk, P.ws->splitk_cap);
  Sweep sw(P, oo);
  sw.ir_inner = o.ir_max > 0;
  sw.upload_initial();
  sw.reverse();
  sw.qr_pass();
  sw.reverse();
  int sweeps = 0, sweeps_total = 0;
  double last = INFINITY;
  int converged = 0;
  // half-sweeps until the local residuals meet tol or the budget is spent
  auto run_sweeps = [&](int budget, const char* what) {
    int done = 0;
    converged = 0;
    for (; done < budget;) {
      last = sw.half_sweep();
      ++done;
      ++sweeps_total;
      if (verbose) {
        const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        std::string rk;
        for (int r : sw.xr) rk += std::to_string(r) + " ";
        fprintf(stderr, "[tnfem] %s half-sweep %d max_res %.3e cg %lld t %.3fs ranks %s\n", what, done, last,
                sw.cg_iters, el, rk.c_str());
      }
      if (sw.nan_seen || !std::isfinite(last)) break;
      sw.reverse();
      if (last <= o.tol) {
        converged = 1;
        break;
      }
    }
    return done;
  };
  sweeps = run_sweeps(o.max_sweeps, "solve");
  int ir_iters = 0;
  double ir_update = 0.0;
  if (o.ir_max > 0 && !sw.nan_seen && std::isfinite(last)) {
    // outer refinement: correction solves on b - A u, u <- round(u + d) in FP64
    P.ensure_ir(o.rank_cap, rho);
    const double ir_tol = o.ir_tol > 0 ? o.ir_tol : o.tol;
    const int ir_sweeps = o.ir_sweeps > 0 ? o.ir_sweeps : o.max_sweeps;
    for (int it = 1; it <= o.ir_max; ++it) {
      if (sw.orient) sw.reverse();
      sw.begin_correction(*P.ws->ir, o.seed_x + it, o.seed_z + it);
      run_sweeps(ir_sweeps, "correction");
      if (sw.nan_seen || !std::isfinite(last)) break;
      if (sw.orient) sw.reverse();
      ir_update = sw.add_correction(*P.ws->ir, 0.1 * ir_tol, o.rank_cap);
      ir_iters = it;
      if (verbose) fprintf(stderr, "[tnfem] refinement %d: ||d|| / ||u|| = %.3e\n", it, ir_update);
      if (!std::isfinite(ir_update)) {
        sw.nan_seen = 1;
        break;
      }
      if (ir_update <= ir_tol) break;
    }
    if (sw.orient) sw.reverse();
    sw.take_u();
    converged = ir_update <= ir_tol && !sw.nan_seen;
  }
  finish_sweep(P, sw, out);
  const auto t1 = std::chrono::steady_clock::now();
  fill_stats(sw, sweeps, converged, last, std::chrono::duration<double>(t1 - t0).count(), stats);
  stats.ir_iters = ir_iters;
  stats.ir_last_update = ir_update;
  stats.sweeps_total = sweeps_total;
  if (o.profile && P.ws->profile) {
    double fl = 0.0;
    long cnt = 0;
    stats.contraction_ms = P.ws->profile->total_ms(&fl, -1, &cnt);
    stats.contraction_flops = fl;
    stats.contraction_launches = cnt;
    const int kind = o.precision ? PROF_FUSED_LOW : PROF_FUSED;
    stats.apply_kernel_ms = P.ws->profile->total_ms(&fl, kind, &cnt);
    stats.apply_kernel_flops = fl;
    stats.apply_kernel_launches = cnt;
  }
  if (sw.nan_seen || !std::isfinite(last)) return TNFEM_ENAN;
  return converged ? TNFEM_OK : TNFEM_ENOTCONV;
}

int run_solve_batch(std::vector<Problem*>& Ps, const tnfem_solve_opts& o, std::vector<HostTT>& outs,
                    std::vector<tnfem_solve_stats>& stats, std::vector<int>& rcs) {
  check_opts(o);
  const int nb = (int)Ps.size();
  TNFEM_REQUIRE(nb >= 1 && nb <= FB_MAX, "a batch holds 1 .. %d problems", FB_MAX);
  TNFEM_REQUIRE(o.ir_max == 0, "batched solves do not run the outer refinement");
  TNFEM_REQUIRE(!o.profile, "batched solves do not record per-launch profiles");
  Context* ctx = Ps[0]->ctx;
  for (Problem* P : Ps) {
    TNFEM_REQUIRE(P->ctx == ctx, "all problems of a batch must share one context");
    TNFEM_REQUIRE(P->K == Ps[0]->K && P->modes == Ps[0]->modes,
                  "all problems of a batch must have the same dimension and level");
  }
  hip_check(hipSetDevice(ctx->device), "hipSetDevice");
  const auto t0 = std::chrono::steady_clock::now();
  tnfem_solve_opts oo = o;
  oo.rho = std::max(o.rho, 1);
  struct Unset {
    ~Unset() { set_gemm_splitk_buffer(nullptr, 0); }
  } unset;
  std::vector<std::unique_ptr<Sweep>> sweeps;
  for (Problem* P : Ps) {
    prepare_workspace(*P, o);
    set_gemm_splitk_buffer(P->ws->splitk, P->ws->splitk_cap);
    auto sw = std::make_unique<Sweep>(*P, oo);
    sw->upload_initial();
    sw->reverse();
    sw->qr_pass();
    sw->reverse();
    sweeps.push_back(std::move(sw));
  }
  BatchArgs args(nb, ctx->allocator);
  outs.assign(nb, HostTT{});
  stats.assign(nb, tnfem_solve_stats{});
  rcs.assign(nb, TNFEM_ENOTCONV);
  std::vector<int> nsw(nb, 0), conv(nb, 0);
  std::vector<double> last(nb, INFINITY);
  std::vector<int> active(nb);
  for (int r = 0; r < nb; ++r) active[r] = r;
  const int K = Ps[0]->K;
  auto finish = [&](int r) {
    finish_sweep(*Ps[r], *sweeps[r], outs[r]);
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    fill_stats(*sweeps[r], nsw[r], conv[r], last[r], secs, stats[r]);
    rcs[r] = (sweeps[r]->nan_seen || !std::isfinite(last[r])) ? TNFEM_ENAN : (conv[r] ? TNFEM_OK : TNFEM_ENOTCONV);
  };
  for (int it = 0; it < o.max_sweeps && !active.empty(); ++it) {
    std::vector<double> mr(nb, 0.0);
    std::vector<int> live = active;
    for (int k = 0; k < K && !live.empty(); ++k) {
      std::vector<Sweep*> S;
      for (int r : live) S.push_back(sweeps[r].get());
      const std::vector<double> res = batch_solve_core(S, k, args, ctx->stream);
      std::vector<int> keep;
      for (size_t i = 0; i < live.size(); ++i) {
        const int r = live[i];
        mr[r] = std::max(mr[r], res[i]);
        if (sweeps[r]->nan_seen) {
          mr[r] = NAN;
          continue;
        }
        keep.push_back(r);
      }
      live.swap(keep);
      if (k < K - 1 && !live.empty()) {
        // truncation and enrichment with shared QR / SVD launches over the requests
        std::vector<Sweep::TruncState> ts(live.size());
        std::vector<QrJob> qj, qj2;
        std::vector<SvdJob> sj;
        for (size_t i = 0; i < live.size(); ++i) {
          const int r = live[i];
          set_gemm_splitk_buffer(Ps[r]->ws->splitk, Ps[r]->ws->splitk_cap);
          sweeps[r]->trunc_begin(k, ts[i]);
          qj.push_back(ts[i].qr);
          sj.push_back(ts[i].svd);
        }
        launch_qr_batch(qj, ctx->stream);
        launch_jacobi_svd_batch(sj, ctx->stream);
        for (size_t i = 0; i < live.size(); ++i) {
          const int r = live[i];
          set_gemm_splitk_buffer(Ps[r]->ws->splitk, Ps[r]->ws->splitk_cap);
          sweeps[r]->trunc_rank(k, ts[i]);
        }
        hip_check(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
        for (size_t i = 0; i < live.size(); ++i) {
          const int r = live[i];
          set_gemm_splitk_buffer(Ps[r]->ws->splitk, Ps[r]->ws->splitk_cap);
          sweeps[r]->enrich_begin(k, ts[i]);
          Sweep::push_enrich_jobs(ts[i], qj2);
        }
        launch_qr_batch(qj2, ctx->stream);
        for (size_t i = 0; i < live.size(); ++i) {
          const int r = live[i];
          set_gemm_splitk_buffer(Ps[r]->ws->splitk, Ps[r]->ws->splitk_cap);
          sweeps[r]->enrich_end(k, ts[i]);
        }
      }
    }
    std::vector<int> still;
    for (int r : active) {
      ++nsw[r];
      last[r] = mr[r];
      Sweep& w = *sweeps[r];
      if (w.nan_seen || !std::isfinite(last[r])) {
        finish(r);
        continue;
      }
      w.reverse();
      if (last[r] <= o.tol) {
        conv[r] = 1;
        finish(r);
        continue;
      }
      still.push_back(r);
    }
    active.swap(still);
  }
  for (int r : active) finish(r);
  return TNFEM_OK;
}

}  // namespace tnfem
