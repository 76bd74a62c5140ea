// Device kernels of the QTT sweep for gfx950 (CDNA4, 64-wide wavefronts).
//
// * gemm_grouped: every contraction of the sweep (local operator apply, local
//   right-hand sides, interface updates, residual projections, core products) is
//   a sum of small matrix products selected by term lists built from the sparse
//   structure of the operator cores.  One kernel evaluates them with FP64 MFMA
//   (v_mfma_f64_16x16x4f64), tiles staged k-major through LDS.
// * Local conjugate gradients keep every scalar on the device; reductions are
//   single-pass (per-block partials, the last block to finish reduces them in a
//   fixed order, so results do not depend on timing).
// * Householder QR and one-sided Jacobi SVD run in one workgroup each; the
//   matrices are at most (r n) x (r + rho) and (r + rho)^2.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <mutex>
#include <cmath>

#include "kernels.hpp"

namespace tnfem {

typedef double d4_t __attribute__((ext_vector_type(4)));

#define TN_CHECK_LAUNCH()                                                                  \
  do {                                                                                     \
    hipError_t e_ = hipGetLastError();                                                     \
    if (e_ != hipSuccess) throw Error(TNFEM_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e_)); \
  } while (0)

}  // namespace tnfem

#include "common.hpp"

namespace tnfem {

// ----------------------------------------------------------------------------- reductions

// Lane exchanges within rows of 16 lanes through DPP (no LDS round trip).  The
// patterns are symmetric, so after each step every lane of a group holds the
// same value, summed in the same order.  All lanes of a group must be active.
enum : int {
  DPP_XOR1 = 0xB1,         // quad_perm [1, 0, 3, 2]
  DPP_XOR2 = 0x4E,         // quad_perm [2, 3, 0, 1]
  DPP_HALF_MIRROR = 0x141, // lane l <- 7 - l within each 8 lanes
  DPP_MIRROR = 0x140,      // lane l <- 15 - l within each 16 lanes
};

template <int CTRL>
__device__ inline double dpp_get(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

__device__ inline double lane_get(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Sum over the 16 lanes of each row.
__device__ inline double row_sum(double v) {
  v += dpp_get<DPP_XOR1>(v);
  v += dpp_get<DPP_XOR2>(v);
  v += dpp_get<DPP_HALF_MIRROR>(v);
  v += dpp_get<DPP_MIRROR>(v);
  return v;
}

// Sum over the wavefront; every lane receives the same value.
__device__ inline double wave_sum(double v) {
  v = row_sum(v);
  return (lane_get(v, 0) + lane_get(v, 16)) + (lane_get(v, 32) + lane_get(v, 48));
}

// Sum over a group of `width` consecutive lanes (width a power of two <= 64, groups aligned).
__device__ inline double group_sum(double v, int width) {
  if (width >= 2) v += dpp_get<DPP_XOR1>(v);
  if (width >= 4) v += dpp_get<DPP_XOR2>(v);
  if (width >= 8) v += dpp_get<DPP_HALF_MIRROR>(v);
  if (width >= 16) v += dpp_get<DPP_MIRROR>(v);
  if (width >= 32) v += __shfl_xor(v, 16, 64);
  if (width >= 64) v += __shfl_xor(v, 32, 64);
  return v;
}

template <int NT>
__device__ inline double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < NT / 64; ++i) s += red[i];
  return s;
}

// ----------------------------------------------------------------------------- grouped GEMM

struct GemmArgs {
  const double* A;
  long a_slot, a_sm, a_sk;
  const double* B;
  long b_slot, b_sk, b_sn;
  double* C;
  long c_slot, c_sm, c_sn;
  int M, N, K;
  const int* grp_beg;
  const int* grp_c;
  const int* t_a;
  const int* t_b;
  const double* t_v;
  double alpha, beta;
  const int* skip;
  int tiles_n, ntiles, ngroups, ksplit;
  double* partial;
};

constexpr int BK = 32;

// 4 waves in a 2 x 2 arrangement; each wave owns WMB x WNB blocks of 16 x 16.
// blockIdx.x: output tile, blockIdx.y: group, blockIdx.z: split of the group's
// (term, k-step) iterations.
template <int WMB, int WNB>
__device__ __forceinline__ void gemm_body(const GemmArgs& g, const int tile, const int grp, const int z) {
  constexpr int TM = 32 * WMB, TN = 32 * WNB;
  __shared__ double sA[BK][TM + 1];
  __shared__ double sB[BK][TN + 1];
  if (g.skip && *g.skip) return;
  const int m0 = (tile / g.tiles_n) * TM, n0 = (tile % g.tiles_n) * TN;
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int wm = wave / 2, wn = wave % 2;
  const int lrow = lane % 16, lk = lane / 16;

  int tb, te;
  if (g.grp_beg) {
    tb = g.grp_beg[grp];
    te = g.grp_beg[grp + 1];
  } else {
    tb = grp;
    te = grp + 1;
  }
  const int nks = (g.K + BK - 1) / BK;
  const long iters = (long)(te - tb) * nks;
  const long chunk = (iters + g.ksplit - 1) / g.ksplit;
  const long it0 = (long)z * chunk;
  const long it1 = it0 + chunk < iters ? it0 + chunk : iters;

  d4_t acc[WMB][WNB];
  for (int i = 0; i < WMB; ++i)
    for (int j = 0; j < WNB; ++j) acc[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};

  const bool a_kfast = (g.a_sk == 1);
  const bool b_nfast = (g.b_sn == 1);
  // thread -> NA elements of the A tile and NB of the B tile, idx = tid + 256 u
  constexpr int NA = TM * BK / 256, NB = TN * BK / 256;
  auto a_pos = [&](int idx, int& mm, int& kk) {
    mm = a_kfast ? idx / BK : idx % TM;
    kk = a_kfast ? idx % BK : idx / TM;
  };
  auto b_pos = [&](int idx, int& nn, int& kk) {
    nn = b_nfast ? idx % TN : idx / BK;
    kk = b_nfast ? idx / TN : idx % BK;
  };
  // the operands of one (term, k-step) iteration into registers: every load issued
  // before any is used (out-of-range elements read the slot's first element and are
  // replaced by zero)
  double ra[NA], rb[NB];
  auto load = [&](long it) {
    const int t = tb + (int)(it / nks);
    const int k0 = (int)(it % nks) * BK;
    const int ai = g.grp_beg ? g.t_a[t] : t;
    const int bi = g.grp_beg ? g.t_b[t] : t;
    const double v = g.t_v ? g.t_v[t] : 1.0;
    const double* Ab = g.A + (long)ai * g.a_slot;
    const double* Bb = g.B + (long)bi * g.b_slot;
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      int mm, kk;
      a_pos(tid + 256 * u, mm, kk);
      const int gm = m0 + mm, gk = k0 + kk;
      const bool in = gm < g.M && gk < g.K;
      const double a = Ab[in ? (long)gm * g.a_sm + (long)gk * g.a_sk : 0];
      ra[u] = in ? v * a : 0.0;
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      int nn, kk;
      b_pos(tid + 256 * u, nn, kk);
      const int gn = n0 + nn, gk = k0 + kk;
      const bool in = gn < g.N && gk < g.K;
      const double b = Bb[in ? (long)gk * g.b_sk + (long)gn * g.b_sn : 0];
      rb[u] = in ? b : 0.0;
    }
  };
  if (it0 < it1) load(it0);
  for (long it = it0; it < it1; ++it) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      int mm, kk;
      a_pos(tid + 256 * u, mm, kk);
      sA[kk][mm] = ra[u];
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      int nn, kk;
      b_pos(tid + 256 * u, nn, kk);
      sB[kk][nn] = rb[u];
    }
    // the next iteration's operands load while this one's products run
    if (it + 1 < it1) load(it + 1);
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      double af[WMB], bf[WNB];
#pragma unroll
      for (int i = 0; i < WMB; ++i) af[i] = sA[kk + lk][wm * 16 * WMB + i * 16 + lrow];
#pragma unroll
      for (int j = 0; j < WNB; ++j) bf[j] = sB[kk + lk][wn * 16 * WNB + j * 16 + lrow];
#pragma unroll
      for (int i = 0; i < WMB; ++i)
#pragma unroll
        for (int j = 0; j < WNB; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  if (g.ksplit > 1) {
    // full (padded) partial tile, row-major TM x TN
    double* Pt = g.partial + (((long)z * g.ngroups + grp) * g.ntiles + tile) * (long)(TM * TN);
    for (int i = 0; i < WMB; ++i)
      for (int j = 0; j < WNB; ++j) {
        const int col = wn * 16 * WNB + j * 16 + lrow;
        for (int q = 0; q < 4; ++q) {
          const int row = wm * 16 * WMB + i * 16 + 4 * q + lk;
          Pt[row * TN + col] = acc[i][j][q];
        }
      }
    return;
  }
  const int ci = g.grp_c ? g.grp_c[grp] : grp;
  double* Cb = g.C + (long)ci * g.c_slot;
  // v_mfma_f64_16x16x4f64 result: D[r][c] is in lane c + 16 (r % 4), register r / 4
  auto c_off = [&](int i, int j, int q, bool& in) {
    const int col = n0 + wn * 16 * WNB + j * 16 + lrow;
    const int row = m0 + wm * 16 * WMB + i * 16 + 4 * q + lk;
    in = row < g.M && col < g.N;
    return in ? (long)row * g.c_sm + (long)col * g.c_sn : 0L;
  };
  // with beta != 0 the old C values are all read before any is written back
  double cv[WMB][WNB][4];
  if (g.beta != 0.0) {
#pragma unroll
    for (int i = 0; i < WMB; ++i)
#pragma unroll
      for (int j = 0; j < WNB; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          bool in;
          cv[i][j][q] = Cb[c_off(i, j, q, in)];
        }
  }
#pragma unroll
  for (int i = 0; i < WMB; ++i)
#pragma unroll
    for (int j = 0; j < WNB; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        bool in;
        const long off = c_off(i, j, q, in);
        if (in) {
          const double val = g.alpha * acc[i][j][q];
          Cb[off] = (g.beta == 0.0) ? val : val + g.beta * cv[i][j][q];
        }
      }
}

// Sums the split partial tiles in split order and writes C (alpha, beta as above).
// One thread per tile element; blockIdx.z covers the tile's elements.
template <int TM, int TN>
__device__ __forceinline__ void splitk_reduce_body(const GemmArgs& g, const int tile, const int grp, const int ez) {
  if (g.skip && *g.skip) return;
  const int e = ez * 256 + threadIdx.x;
  if (e >= TM * TN) return;
  const int m0 = (tile / g.tiles_n) * TM, n0 = (tile % g.tiles_n) * TN;
  const int row = m0 + e / TN, col = n0 + e % TN;
  if (row >= g.M || col >= g.N) return;
  const long stride = (long)g.ngroups * g.ntiles * (TM * TN);
  const double* src = g.partial + ((long)grp * g.ntiles + tile) * (long)(TM * TN) + e;
  double s = 0.0;
  int z = 0;
  for (; z + 4 <= g.ksplit; z += 4) {
    const double a0 = src[(long)z * stride], a1 = src[(long)(z + 1) * stride];
    const double a2 = src[(long)(z + 2) * stride], a3 = src[(long)(z + 3) * stride];
    s += a0;
    s += a1;
    s += a2;
    s += a3;
  }
  for (; z < g.ksplit; ++z) s += src[(long)z * stride];
  const int ci = g.grp_c ? g.grp_c[grp] : grp;
  double* c = g.C + (long)ci * g.c_slot + (long)row * g.c_sm + (long)col * g.c_sn;
  const double val = g.alpha * s;
  *c = (g.beta == 0.0) ? val : val + g.beta * *c;
}

template <int WMB, int WNB>
__global__ __launch_bounds__(256) void gemm_grouped_kernel(GemmArgs g) {
  gemm_body<WMB, WNB>(g, blockIdx.x, blockIdx.y, blockIdx.z);
}

template <int TM, int TN>
__global__ __launch_bounds__(256) void splitk_reduce_kernel(GemmArgs g) {
  splitk_reduce_body<TM, TN>(g, blockIdx.x, blockIdx.y, blockIdx.z);
}

// Several independent grouped GEMMs of one tile class in one launch: the flattened
// grid is cut into consecutive ranges, one per descriptor, each walked in the
// (tile, group, split) order of the single launch (and, for the split sums, the
// (tile, group, element block) order).
constexpr int GM_MAX = 6;
struct GemmMulti {
  GemmArgs g[GM_MAX];
  int beg[GM_MAX + 1];
  int n;
};

__device__ __forceinline__ int multi_find(const GemmMulti& m, int b) {
  int d = 0;
  while (d + 1 < m.n && b >= m.beg[d + 1]) ++d;
  return d;
}

template <int WMB, int WNB>
__global__ __launch_bounds__(256) void gemm_multi_kernel(GemmMulti m) {
  const int d = multi_find(m, blockIdx.x);
  const GemmArgs& g = m.g[d];
  const int loc = blockIdx.x - m.beg[d];
  const int per = g.ntiles * g.ngroups;
  const int z = loc / per, rem = loc - z * per;
  const int grp = rem / g.ntiles;
  gemm_body<WMB, WNB>(g, rem - grp * g.ntiles, grp, z);
}

template <int TM, int TN>
__global__ __launch_bounds__(256) void splitk_reduce_multi_kernel(GemmMulti m) {
  const int d = multi_find(m, blockIdx.x);
  const GemmArgs& g = m.g[d];
  const int loc = blockIdx.x - m.beg[d];
  const int per = g.ntiles * g.ngroups;
  const int ez = loc / per, rem = loc - ez * per;
  const int grp = rem / g.ntiles;
  splitk_reduce_body<TM, TN>(g, rem - grp * g.ntiles, grp, ez);
}

static thread_local GemmProfile* g_prof = nullptr;
static thread_local int g_prof_tag = -1;
void set_gemm_profile(GemmProfile* p) { g_prof = p; }
void set_profile_tag(int tag) { g_prof_tag = tag; }
size_t profile_mark() { return g_prof ? g_prof->used : 0; }
void profile_drop_from(size_t mark, int min_tag) {
  GemmProfile* p = g_prof;
  if (!p) return;
  for (size_t i = mark; i < p->used; ++i)
    if (p->tag[i] >= min_tag) p->valid[i] = 0;
}
static thread_local double* g_splitk = nullptr;
static thread_local size_t g_splitk_cap = 0;
void set_gemm_splitk_buffer(double* p, size_t cap) {
  g_splitk = p;
  g_splitk_cap = p ? cap : 0;
}

GemmProfile::~GemmProfile() {
  for (hipEvent_t e : ev) (void)hipEventDestroy(e);
}

double GemmProfile::total_ms(double* total_flops, int want, long* launches) {
  double ms = 0.0, fl = 0.0;
  long cnt = 0;
  if (used > 0) (void)hipEventSynchronize(ev[2 * used - 1]);
  for (size_t i = 0; i < used; ++i) {
    if (want >= 0 && kind[i] != want) continue;
    float t = 0.0f;
    if (hipEventElapsedTime(&t, ev[2 * i], ev[2 * i + 1]) == hipSuccess) ms += t;
    if (valid[i]) fl += flops[i];
    ++cnt;
  }
  if (total_flops) *total_flops = fl;
  if (launches) *launches = cnt;
  return ms;
}

static void launch_gemm_impl(const GemmDesc& d, hipStream_t s);

void launch_gemm(const GemmDesc& d, hipStream_t s) {
  if (d.M <= 0 || d.N <= 0 || d.ngroups <= 0) return;
  launch_gemm_impl(d, s);
}

// Event pair around the contraction kernel itself (not its split-K reduction).
static hipEvent_t* prof_begin(hipStream_t s) {
  GemmProfile* p = g_prof;
  if (!p || p->used >= p->limit) return nullptr;
  while (p->ev.size() < 2 * (p->used + 1)) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) throw Error(TNFEM_EDEVICE, "hipEventCreate");
    p->ev.push_back(e);
  }
  return &p->ev[2 * p->used];
}

// Launch; with a profile pair, the dispatch itself stamps the pair with the kernel's
// start and end (the same timestamps a kernel trace reports).
#define TN_LAUNCH(ev, kernel, grid, block, shm, s, ...)                                      \
  do {                                                                                   \
    if (ev)                                                                              \
      hipExtLaunchKernelGGL(kernel, grid, block, shm, s, (ev)[0], (ev)[1], 0, __VA_ARGS__); \
    else                                                                                 \
      hipLaunchKernelGGL(kernel, grid, block, shm, s, __VA_ARGS__);                      \
  } while (0)

static void prof_end(hipEvent_t* pair, double flops, hipStream_t s, int kind) {
  (void)s;
  if (!pair) return;
  g_prof->flops.push_back(flops);
  g_prof->kind.push_back(kind);
  g_prof->tag.push_back(g_prof_tag);
  g_prof->valid.push_back(1);
  g_prof->used++;
}

// Workgroups wanted per launch before splitting is considered (256 CUs).
constexpr long SPLIT_TARGET_WG = 512;
constexpr int SPLIT_MIN_ITERS = 2;  // (term, k-step) iterations per split at least

static GemmArgs gemm_args(const GemmDesc& d) {
  return GemmArgs{d.A, d.a_slot, d.a_sm, d.a_sk, d.B, d.b_slot, d.b_sk, d.b_sn, d.C, d.c_slot, d.c_sm, d.c_sn,
                  d.M, d.N, d.K, d.grp_beg, d.grp_c, d.t_a, d.t_b, d.t_v, d.alpha, d.beta, d.skip, 0, 0, 0, 1, nullptr};
}

// Tile counts and the split of a descriptor's (term, k-step) iterations; the partial
// tiles go to pbuf (pcap doubles free there).  Returns the doubles of partials used.
template <int WMB, int WNB>
static size_t plan_tiled(GemmArgs& a, const GemmDesc& d, double* pbuf, size_t pcap) {
  constexpr int TM = 32 * WMB, TN = 32 * WNB;
  a.tiles_n = (d.N + TN - 1) / TN;
  a.ntiles = ((d.M + TM - 1) / TM) * a.tiles_n;
  a.ngroups = d.ngroups;
  a.ksplit = 1;
  a.partial = pbuf;
  const long natural = (long)a.ntiles * d.ngroups;
  const long iters = (long)std::max(d.max_terms, 1) * ((d.K + BK - 1) / BK);
  if (pbuf && natural < SPLIT_TARGET_WG && iters >= 2 * SPLIT_MIN_ITERS) {
    long ks = (SPLIT_TARGET_WG + natural - 1) / natural;
    ks = std::min(ks, iters / SPLIT_MIN_ITERS);
    const long per = natural * (long)(TM * TN);
    ks = std::min(ks, (long)(pcap / std::max(per, 1L)));
    ks = std::min(ks, 64L);
    if (ks >= 2) a.ksplit = (int)ks;
  }
  return a.ksplit > 1 ? (size_t)natural * a.ksplit * (TM * TN) : 0;
}

template <int WMB, int WNB>
static void launch_tiled(GemmArgs a, const GemmDesc& d, hipStream_t s) {
  constexpr int TM = 32 * WMB, TN = 32 * WNB;
  if (d.partial) plan_tiled<WMB, WNB>(a, d, d.partial, d.partial_cap);
  else plan_tiled<WMB, WNB>(a, d, g_splitk, g_splitk_cap);
  dim3 grid(a.ntiles, d.ngroups, a.ksplit);
  hipEvent_t* ev = prof_begin(s);
  TN_LAUNCH(ev, (gemm_grouped_kernel<WMB, WNB>), grid, dim3(256), 0, s, a);
  prof_end(ev, d.flops, s, PROF_GEMM);
  TN_CHECK_LAUNCH();
  if (a.ksplit > 1) {
    hipLaunchKernelGGL((splitk_reduce_kernel<TM, TN>), dim3(a.ntiles, d.ngroups, (TM * TN + 255) / 256), dim3(256), 0,
                       s, a);
    TN_CHECK_LAUNCH();
  }
}

static bool gemm_wide(const GemmDesc& d) { return d.M >= 64 && d.N >= 64; }

static void launch_gemm_impl(const GemmDesc& d, hipStream_t s) {
  const GemmArgs a = gemm_args(d);
  if (gemm_wide(d)) launch_tiled<2, 2>(a, d, s);
  else launch_tiled<1, 1>(a, d, s);
}

// One launch for the descriptors of one tile class (at most GM_MAX), the split sums of
// those that split in a second one.  Each descriptor splits as it would alone, its
// partial tiles in its own part of the split-K buffer (fewer splits where the buffer
// runs out), so every result equals the one of its own launch.
template <int WMB, int WNB>
static void launch_multi_class(const GemmDesc* ds, const int* idx, int n, hipStream_t s) {
  constexpr int TM = 32 * WMB, TN = 32 * WNB;
  GemmMulti m{};
  GemmMulti r{};
  m.n = r.n = n;
  size_t used = 0;
  long wg = 0, rwg = 0;
  double flops = 0.0;
  bool any_split = false;
  for (int j = 0; j < n; ++j) {
    const GemmDesc& d = ds[idx[j]];
    GemmArgs a = gemm_args(d);
    if (d.partial) {
      plan_tiled<WMB, WNB>(a, d, d.partial, d.partial_cap);
    } else {
      double* pbuf = g_splitk ? g_splitk + used : nullptr;
      used += plan_tiled<WMB, WNB>(a, d, pbuf, g_splitk ? g_splitk_cap - used : 0);
    }
    m.g[j] = r.g[j] = a;
    m.beg[j] = (int)wg;
    r.beg[j] = (int)rwg;
    wg += (long)a.ntiles * a.ngroups * a.ksplit;
    if (a.ksplit > 1) {
      rwg += (long)a.ntiles * a.ngroups * ((TM * TN + 255) / 256);
      any_split = true;
    }
    flops += d.flops;
  }
  m.beg[n] = (int)wg;
  r.beg[n] = (int)rwg;
  if (wg > INT32_MAX / 2) throw Error(TNFEM_EINVAL, "grouped GEMM launch too large");
  hipEvent_t* ev = prof_begin(s);
  TN_LAUNCH(ev, (gemm_multi_kernel<WMB, WNB>), dim3((unsigned)wg), dim3(256), 0, s, m);
  prof_end(ev, flops, s, PROF_GEMM);
  TN_CHECK_LAUNCH();
  if (any_split) {
    hipLaunchKernelGGL((splitk_reduce_multi_kernel<TM, TN>), dim3((unsigned)rwg), dim3(256), 0, s, r);
    TN_CHECK_LAUNCH();
  }
}

void launch_gemm_multi(const GemmDesc* ds, int n, hipStream_t s) {
  int wide[GM_MAX], narrow[GM_MAX];
  int nw = 0, nn = 0;
  auto flush = [&]() {
    if (nw == 1) launch_gemm_impl(ds[wide[0]], s);
    else if (nw > 1) launch_multi_class<2, 2>(ds, wide, nw, s);
    if (nn == 1) launch_gemm_impl(ds[narrow[0]], s);
    else if (nn > 1) launch_multi_class<1, 1>(ds, narrow, nn, s);
    nw = nn = 0;
  };
  for (int i = 0; i < n; ++i) {
    const GemmDesc& d = ds[i];
    if (d.M <= 0 || d.N <= 0 || d.ngroups <= 0) continue;
    if (gemm_wide(d)) wide[nw++] = i;
    else narrow[nn++] = i;
    if (nw == GM_MAX || nn == GM_MAX) flush();
  }
  flush();
}

// ----------------------------------------------------------------------------- CG

constexpr int CG_MAXB = 512;

// ----------------------------------------------------------------------------- fused local apply

// y partial tiles for a sparse operator core (every term a product of small blocks):
//   part[z][i'][tile][32 x 32] = sum_{terms (slot, e, v) of group i' in split z}
//                                v (L[rows, b, :] x[:, i, :]) Rt[cols, e, :]^T
// The stage-1 product (rows of T1 = L_b x_i for this tile) is formed in LDS per
// term and consumed at once.  Padded rows/cols are written as zeros.
// Operand precision of the fused apply: 0 = FP64 operands and accumulation
// (v_mfma_f64_16x16x4f64), 1 = FP32 operands, FP32 accumulation
// (v_mfma_f32_16x16x4f32), 2 = BF16 operands, FP32 accumulation
// (v_mfma_f32_16x16x32_bf16).  Inputs are FP64 in memory and rounded when staged;
// the stage-1 product is rounded to the operand type before stage 3; partial
// tiles are written as FP64.
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

// Sum of one value per thread over a 256-thread workgroup in a fixed order, stored by
// thread 0 (every thread of the workgroup must call it).
__device__ inline void store_block_dot(double d, double* dst) {
  __shared__ double red[4];
  d = wave_sum(d);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x / 64] = d;
  __syncthreads();
  if (threadIdx.x == 0) *dst = (red[0] + red[1]) + (red[2] + red[3]);
}

template <int P>
struct Prec;
template <>
struct Prec<0> {
  using T = double;
  using Acc = d4_t;
};
template <>
struct Prec<1> {
  using T = float;
  using Acc = f4_t;
};
template <>
struct Prec<2> {
  using T = __bf16;
  using Acc = f4_t;
};

// Row (within a 16 x 16 block) held by accumulator entry q of lane (lk = lane / 16).
template <int P>
__device__ inline int acc_row(int q, int lk) {
  return P == 0 ? 4 * q + lk : 4 * lk + q;
}

// acc += A[arow + 0..15][0..31] * B[0..31][bcol + 0..15], A stored sA[k][m], B stored sB[k][n].
template <int P>
__device__ inline void mfma_k32(const typename Prec<P>::T (*sA)[33], const typename Prec<P>::T (*sB)[33], int arow,
                                int bcol, int lk, int lrow, typename Prec<P>::Acc& acc) {
  if constexpr (P == 0) {
#pragma unroll
    for (int kk = 0; kk < 32; kk += 4)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(sA[kk + lk][arow + lrow], sB[kk + lk][bcol + lrow], acc, 0, 0, 0);
  } else if constexpr (P == 1) {
#pragma unroll
    for (int kk = 0; kk < 32; kk += 4)
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(sA[kk + lk][arow + lrow], sB[kk + lk][bcol + lrow], acc, 0, 0, 0);
  } else {
    bf8_t a, b;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      a[j] = sA[8 * lk + j][arow + lrow];
      b[j] = sB[8 * lk + j][bcol + lrow];
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
  }
}

// The same on LDS tiles of row length LD, over k = k0 .. k0 + 31.
template <int P, int LD>
__device__ inline void mfma_k32o(const typename Prec<P>::T (*sA)[LD], const typename Prec<P>::T (*sB)[LD], int k0,
                                 int arow, int bcol, int lk, int lrow, typename Prec<P>::Acc& acc) {
  if constexpr (P == 0) {
#pragma unroll
    for (int kk = 0; kk < 32; kk += 4)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(sA[k0 + kk + lk][arow + lrow], sB[k0 + kk + lk][bcol + lrow], acc, 0,
                                                 0, 0);
  } else if constexpr (P == 1) {
#pragma unroll
    for (int kk = 0; kk < 32; kk += 4)
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(sA[k0 + kk + lk][arow + lrow], sB[k0 + kk + lk][bcol + lrow], acc, 0,
                                                 0, 0);
  } else {
    bf8_t a, b;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      a[j] = sA[k0 + 8 * lk + j][arow + lrow];
      b[j] = sB[k0 + 8 * lk + j][bcol + lrow];
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
  }
}

// Raw buffer over n doubles from base: loads beyond the range read zero, and one offset
// register serves all the loads of a tile (the rest of each offset in the scalar field).
__device__ inline __amdgpu_buffer_rsrc_t tile_rsrc(const double* base, long n) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(base), (short)0, (int)(n * 8), 0x00020000);
}
__device__ inline double tile_load(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

// Term metadata of a workgroup's term range tb .. te - 1, read once into the lanes:
// lane l of every wavefront holds term tb + l (l < 64); terms beyond are read directly.
// (code: f.tc for the one-pass kernels, f.ta (slot) for the two-stage apply)
__device__ inline void term_prefetch(const FusedArgs& f, const int* code, int tb, int te, int lane, int& mc, int& me,
                                     double& mv) {
  const int t = tb + lane;
  const bool ok = t < te;
  mc = ok ? code[t] : 0;
  me = ok ? f.tb[t] : 0;
  mv = ok ? f.tv[t] : 0.0;
}

__device__ inline void term_get(const FusedArgs& f, const int* codes, int t, int tb, int mc, int me, double mv,
                                int& code, int& e, double& v) {
  const int j = t - tb;
  if (j < 64) {
    code = __builtin_amdgcn_readlane(mc, j);
    e = __builtin_amdgcn_readlane(me, j);
    const long long bits = __double_as_longlong(mv);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(bits & 0xffffffffLL), j);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(bits >> 32), j);
    v = __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
  } else {
    code = codes[t];
    e = f.tb[t];
    v = f.tv[t];
  }
}

// The fused apply for 32 < max(p, q, s, t) <= 64: one workgroup computes the whole
// p x t output of its mode (each wave one 32 x 32 quadrant), so the stage-1 product
// L_b x_i (p x s, K = q) is formed once per term; the next term's operands are
// loaded into registers while the current term's products run.  Partial tiles are
// written in the 32 x 32 tile layout of the general kernel.
// Two workgroups of the one-pass applies share a compute unit (two LDS tiles each, at
// most 256 registers a lane), so one's loads and barriers overlap the other's products.
#define FUSED2_OCC __attribute__((amdgpu_waves_per_eu(2)))

template <int P>
__device__ __forceinline__ void fused_apply64_body(const FusedArgs& f, const int grp, const int z) {
  using T = typename Prec<P>::T;
  using Acc = typename Prec<P>::Acc;
  __shared__ T sA[64][65];  // stage 1: L rows (sA[k][m]); stage 2: Rt^T (sA[s][t])
  __shared__ T sB[64][65];  // stage 1: x (sB[k][n]); stage 2: the stage-1 product (sB[s][p])
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int wm = wave / 2, wn = wave % 2;
  const int lrow = lane % 16, lk = lane / 16;
  const int tb0 = f.begv[grp], te0 = f.begv[grp + 1];
  const int cnt = te0 - tb0;
  const int chunk = (cnt + f.ksplit - 1) / f.ksplit;
  const int tb = tb0 + z * chunk;
  const int te = tb + chunk < te0 ? tb + chunk : te0;
  const long Lrow = (long)f.Rl * f.q, Xrow = (long)f.n * f.s, Rrow = (long)f.Rr * f.s;
  // the term metadata and the skip flag are read together, before any tile load
  int mc, me;
  double mv;
  term_prefetch(f, f.tc, tb, te, lane, mc, me, mv);
  if (f.skip && *f.skip) return;
  double la[16], xb[16], rb[16], vcur = 0.0;
  // thread -> rows tid / 64 + 4 j, column tid % 64 of each tile: rows beyond the tile's
  // row count lie beyond the buffer range, and so does every offset of a column beyond
  // it (both read zero without a memory access)
  const int r0 = tid / 64, c0 = tid % 64;
  const bool cq = c0 < f.q, cs = c0 < f.s;
  constexpr int OUT = 0x40000000;
  const double* re_next = nullptr;
  auto load_lx = [&](int t, double& v) {
    int code, e;
    term_get(f, f.tc, t, tb, mc, me, mv, code, e, v);
    const long lb = (long)(code >> 4) * f.q, xi = (long)(code & 15) * f.s;
    re_next = f.Rt + (long)e * f.s;
    const __amdgpu_buffer_rsrc_t rl = tile_rsrc(f.L + lb, (long)f.p * Lrow - lb);
    const __amdgpu_buffer_rsrc_t rx = tile_rsrc(f.x + xi, (long)f.q * Xrow - xi);
    const int vl = cq ? (int)((r0 * Lrow + c0) * 8) : OUT, vx = cs ? (int)((r0 * Xrow + c0) * 8) : OUT;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      la[j] = tile_load(rl, vl, (int)(4 * j * Lrow * 8));
      xb[j] = tile_load(rx, vx, (int)(4 * j * Xrow * 8));
    }
  };
  auto load_r = [&](const double* Re) {
    const long re = Re - f.Rt;
    const __amdgpu_buffer_rsrc_t rt = tile_rsrc(Re, (long)f.t * Rrow - re);
    const int vr = cs ? (int)((r0 * Rrow + c0) * 8) : OUT;
#pragma unroll
    for (int j = 0; j < 16; ++j) rb[j] = tile_load(rt, vr, (int)(4 * j * Rrow * 8));
  };
  if (tb < te) {
    load_lx(tb, vcur);
    load_r(re_next);
  }
  Acc acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = Acc{0, 0, 0, 0};
  for (int t = tb; t < te; ++t) {
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int idx = tid + 256 * j, r = idx / 64, c = idx % 64;
      sA[c][r] = (T)la[j];  // A = L rows (m = r) x q (k = c)
      sB[r][c] = (T)xb[j];  // B = x (k = r) x s (n = c)
    }
    const double v = vcur;
    const bool more = t + 1 < te;
    if (more) load_lx(t + 1, vcur);
    __syncthreads();
    Acc tacc[2][2];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int ni = 0; ni < 2; ++ni) {
        tacc[mi][ni] = Acc{0, 0, 0, 0};
        mfma_k32o<P, 65>(sA, sB, 0, wm * 32 + mi * 16, wn * 32 + ni * 16, lk, lrow, tacc[mi][ni]);
        mfma_k32o<P, 65>(sA, sB, 32, wm * 32 + mi * 16, wn * 32 + ni * 16, lk, lrow, tacc[mi][ni]);
      }
    __syncthreads();
    // stage 2 operands into the same tiles: the stage-1 product and Rt^T
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int ni = 0; ni < 2; ++ni)
#pragma unroll
        for (int qq = 0; qq < 4; ++qq)
          sB[wn * 32 + ni * 16 + lrow][wm * 32 + mi * 16 + acc_row<P>(qq, lk)] = (T)(v * (double)tacc[mi][ni][qq]);
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int idx = tid + 256 * j, r = idx / 64, c = idx % 64;
      sA[c][r] = (T)rb[j];  // B' = Rt^T: k = s (c), n = t (r)
    }
    if (more) load_r(re_next);
    __syncthreads();
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int ni = 0; ni < 2; ++ni) {
        mfma_k32o<P, 65>(sB, sA, 0, wm * 32 + mi * 16, wn * 32 + ni * 16, lk, lrow, acc[mi][ni]);
        mfma_k32o<P, 65>(sB, sA, 32, wm * 32 + mi * 16, wn * 32 + ni * 16, lk, lrow, acc[mi][ni]);
      }
    __syncthreads();
  }
  // quadrant (wm, wn) is the 32 x 32 tile (wm, wn) of the general layout, when it exists
  if (wm * 32 < f.p && wn * 32 < f.t) {
    const int tile = wm * f.tiles_n + wn;
    double* Pt = f.partial + (((long)z * f.n + grp) * f.ntiles + tile) * 1024;
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int ni = 0; ni < 2; ++ni)
#pragma unroll
        for (int qq = 0; qq < 4; ++qq)
          Pt[(mi * 16 + acc_row<P>(qq, lk)) * 32 + ni * 16 + lrow] = (double)acc[mi][ni][qq];
  }
  if (f.dots) {
    // x at the fragment positions: all loads issued together (out-of-range positions read
    // element 0 and are not added), then summed in fragment order
    double xv[2][2][4];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int ni = 0; ni < 2; ++ni)
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
          const int row = wm * 32 + mi * 16 + acc_row<P>(qq, lk), col = wn * 32 + ni * 16 + lrow;
          const bool in = row < f.p && col < f.t;
          xv[mi][ni][qq] = f.x[in ? ((long)row * f.n + grp) * f.s + col : 0];
        }
    double d = 0.0;
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int ni = 0; ni < 2; ++ni)
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
          const int row = wm * 32 + mi * 16 + acc_row<P>(qq, lk), col = wn * 32 + ni * 16 + lrow;
          if (row < f.p && col < f.t) d += (double)acc[mi][ni][qq] * xv[mi][ni][qq];
        }
    store_block_dot(d, f.dots + (long)z * f.n + grp);
  }
}

template <int P>
__global__ __launch_bounds__(256) FUSED2_OCC void fused_apply64_kernel(FusedArgs f) {
  fused_apply64_body<P>(f, blockIdx.y, blockIdx.z);
}

// acc[j] += A[r[j] + 0..15][0..K-1] * B[0..K-1][c[j] + 0..15] for the BPW blocks of a
// wave (A stored sA[k][m], B stored sB[k][n]), K a multiple of 8, k ascending per block.
// The fragments of the next two k steps are read from LDS while the current ones
// are multiplied, so the MFMA pipe does not wait for LDS between steps.
template <int P, int BPW>
__device__ __forceinline__ void mfma_blocks(const typename Prec<P>::T (*sA)[65], const typename Prec<P>::T (*sB)[65],
                                            int K, const int (&r)[BPW], const int (&c)[BPW], int lk, int lrow,
                                            typename Prec<P>::Acc (&acc)[BPW]) {
  using T = typename Prec<P>::T;
  T a[2][BPW], b[2][BPW], an[2][BPW], bn[2][BPW];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int j = 0; j < BPW; ++j) {
      a[h][j] = sA[4 * h + lk][r[j] + lrow];
      b[h][j] = sB[4 * h + lk][c[j] + lrow];
    }
  for (int kk = 0; kk < K; kk += 8) {
    const bool more = kk + 8 < K;
    if (more) {
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int j = 0; j < BPW; ++j) {
          an[h][j] = sA[kk + 8 + 4 * h + lk][r[j] + lrow];
          bn[h][j] = sB[kk + 8 + 4 * h + lk][c[j] + lrow];
        }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int j = 0; j < BPW; ++j) {
        if constexpr (P == 0)
          acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[h][j], b[h][j], acc[j], 0, 0, 0);
        else
          acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[h][j], b[h][j], acc[j], 0, 0, 0);
      }
    if (more) {
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int j = 0; j < BPW; ++j) {
          a[h][j] = an[h][j];
          b[h][j] = bn[h][j];
        }
    }
  }
}

// FP64 and FP32 operands, 32 < max(p, q, s, t) <= 64: the same one-pass product on
// 16 x 16 MFMA blocks.  The stage-1 product (p x s) and the output (p x t) are covered
// by ceil(rows / 16) x ceil(cols / 16) blocks and both contractions run over K rounded
// up to 8 (two MFMA depths), so a rank between 33 and 63 costs in proportion to its
// size rather than to 64 (the zero padding adds exact zeros: the results equal those
// of the 64-padded product bit for bit).  Wave w owns blocks w, w + 4, ..., BPW of
// them (slots beyond the block count repeat the last block and are not stored); the
// BPW independent accumulation chains are interleaved per k step.  The stage-1 product
// rows from s to the next multiple of 8 are read by stage 2: stage 1 writes them (zero
// columns of x).
template <int P, int BPW>
__device__ __forceinline__ void fused_apply16_body(const FusedArgs& f, const int grp, const int z) {
  using T = typename Prec<P>::T;
  using Acc = typename Prec<P>::Acc;
  static_assert(P == 0 || P == 1, "16 x 16 x 4 MFMA operands");
  // two tiles for both stages, as in the rank-64 kernel: L and x, then Rt^T and the
  // stage-1 product
  __shared__ T sA[64][65];
  __shared__ T sB[64][65];
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int lrow = lane % 16, lk = lane / 16;
  const int tb0 = f.begv[grp], te0 = f.begv[grp + 1];
  const int cnt = te0 - tb0;
  const int chunk = (cnt + f.ksplit - 1) / f.ksplit;
  const int tb = tb0 + z * chunk;
  const int te = tb + chunk < te0 ? tb + chunk : te0;
  const long Lrow = (long)f.Rl * f.q, Xrow = (long)f.n * f.s, Rrow = (long)f.Rr * f.s;
  int mc, me;
  double mv;
  term_prefetch(f, f.tc, tb, te, lane, mc, me, mv);
  if (f.skip && *f.skip) return;
  const int mb = (f.p + 15) / 16, sbk = (f.s + 15) / 16, tbk = (f.t + 15) / 16;
  const int nb1 = mb * sbk, nb2 = mb * tbk;
  const int k1 = (f.q + 7) & ~7, k2 = (f.s + 7) & ~7;
  // block offsets: stage 1 (rows of p, columns of s), stage 2 (rows of p, columns of t)
  int r1[BPW], c1[BPW], r2[BPW], c2[BPW];
#pragma unroll
  for (int j = 0; j < BPW; ++j) {
    const int b1 = min(wave + 4 * j, nb1 - 1), b2 = min(wave + 4 * j, nb2 - 1);
    r1[j] = (b1 / sbk) * 16;
    c1[j] = (b1 % sbk) * 16;
    r2[j] = (b2 / tbk) * 16;
    c2[j] = (b2 % tbk) * 16;
  }
  double la[16], xb[16], rb[16], vcur = 0.0;
  // thread -> rows tid / 64 + 4 j, column tid % 64 of each tile: rows beyond the tile's
  // row count lie beyond the buffer range, and so does every offset of a column beyond
  // it (both read zero without a memory access)
  const int r0 = tid / 64, c0 = tid % 64;
  const bool cq = c0 < f.q, cs = c0 < f.s;
  constexpr int OUT = 0x40000000;
  const double* re_next = nullptr;
  auto load_lx = [&](int t, double& v) {
    int code, e;
    term_get(f, f.tc, t, tb, mc, me, mv, code, e, v);
    const long lb = (long)(code >> 4) * f.q, xi = (long)(code & 15) * f.s;
    re_next = f.Rt + (long)e * f.s;
    const __amdgpu_buffer_rsrc_t rl = tile_rsrc(f.L + lb, (long)f.p * Lrow - lb);
    const __amdgpu_buffer_rsrc_t rx = tile_rsrc(f.x + xi, (long)f.q * Xrow - xi);
    const int vl = cq ? (int)((r0 * Lrow + c0) * 8) : OUT, vx = cs ? (int)((r0 * Xrow + c0) * 8) : OUT;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      la[j] = tile_load(rl, vl, (int)(4 * j * Lrow * 8));
      xb[j] = tile_load(rx, vx, (int)(4 * j * Xrow * 8));
    }
  };
  auto load_r = [&](const double* Re) {
    const long re = Re - f.Rt;
    const __amdgpu_buffer_rsrc_t rt = tile_rsrc(Re, (long)f.t * Rrow - re);
    const int vr = cs ? (int)((r0 * Rrow + c0) * 8) : OUT;
#pragma unroll
    for (int j = 0; j < 16; ++j) rb[j] = tile_load(rt, vr, (int)(4 * j * Rrow * 8));
  };
  if (tb < te) {
    load_lx(tb, vcur);
    load_r(re_next);
  }
  Acc acc[BPW];
#pragma unroll
  for (int j = 0; j < BPW; ++j) acc[j] = Acc{0, 0, 0, 0};
  for (int t = tb; t < te; ++t) {
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int idx = tid + 256 * j, r = idx / 64, c = idx % 64;
      sA[c][r] = (T)la[j];  // A = L rows (m = r) x q (k = c)
      sB[r][c] = (T)xb[j];  // B = x (k = r) x s (n = c)
    }
    const double v = vcur;
    const bool more = t + 1 < te;
    if (more) load_lx(t + 1, vcur);
    __syncthreads();
    Acc tacc[BPW];
#pragma unroll
    for (int j = 0; j < BPW; ++j) tacc[j] = Acc{0, 0, 0, 0};
    mfma_blocks<P, BPW>(sA, sB, k1, r1, c1, lk, lrow, tacc);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < BPW; ++j) {
      if (wave + 4 * j < nb1) {
#pragma unroll
        for (int qq = 0; qq < 4; ++qq)
          sB[c1[j] + lrow][r1[j] + acc_row<P>(qq, lk)] = (T)(v * (double)tacc[j][qq]);
      }
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int idx = tid + 256 * j, r = idx / 64, c = idx % 64;
      sA[c][r] = (T)rb[j];  // B' = Rt^T: k = s (c), n = t (r)
    }
    if (more) load_r(re_next);
    __syncthreads();
    mfma_blocks<P, BPW>(sB, sA, k2, r2, c2, lk, lrow, acc);
    __syncthreads();
  }
  // block (r2, c2) lies in 32 x 32 tile (r2 / 32, c2 / 32) of the partial layout
#pragma unroll
  for (int j = 0; j < BPW; ++j) {
    if (wave + 4 * j < nb2) {
      double* Pt = f.partial + (((long)z * f.n + grp) * f.ntiles + (r2[j] / 32) * f.tiles_n + c2[j] / 32) * 1024;
#pragma unroll
      for (int qq = 0; qq < 4; ++qq)
        Pt[(r2[j] % 32 + acc_row<P>(qq, lk)) * 32 + c2[j] % 32 + lrow] = (double)acc[j][qq];
    }
  }
  if (f.dots) {
    double xv[BPW][4];
#pragma unroll
    for (int j = 0; j < BPW; ++j)
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        const int row = r2[j] + acc_row<P>(qq, lk), col = c2[j] + lrow;
        const bool in = wave + 4 * j < nb2 && row < f.p && col < f.t;
        xv[j][qq] = f.x[in ? ((long)row * f.n + grp) * f.s + col : 0];
      }
    double d = 0.0;
#pragma unroll
    for (int j = 0; j < BPW; ++j)
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        const int row = r2[j] + acc_row<P>(qq, lk), col = c2[j] + lrow;
        if (wave + 4 * j < nb2 && row < f.p && col < f.t) d += (double)acc[j][qq] * xv[j][qq];
      }
    store_block_dot(d, f.dots + (long)z * f.n + grp);
  }
}

template <int P, int BPW>
__global__ __launch_bounds__(256) FUSED2_OCC void fused_apply16_kernel(FusedArgs f) {
  fused_apply16_body<P, BPW>(f, blockIdx.y, blockIdx.z);
}

// 16 x 16 blocks per wave for the 16-granular apply (stage 1 and the output)
int fused16_bpw(const FusedArgs& f) {
  const int mb = (f.p + 15) / 16;
  const int nb = std::max(mb * ((f.s + 15) / 16), mb * ((f.t + 15) / 16));
  return (nb + 3) / 4;
}

// Fast path of the fused apply for p, q, s, t <= 32 (one tile, one chunk of each
// contracted index): the next term's operand tiles are loaded into registers
// while the current term's two MFMA products run.
template <int P>
__device__ __forceinline__ void fused_apply32_body(const FusedArgs& f, const int grp, const int z) {
  using T = typename Prec<P>::T;
  using Acc = typename Prec<P>::Acc;
  __shared__ T sA[32][33];
  __shared__ T sB[32][33];
  __shared__ T sT[32][33];
  __shared__ T sR[32][33];
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int wm = wave / 2, wn = wave % 2;
  const int lrow = lane % 16, lk = lane / 16;
  const int tb0 = f.begv[grp], te0 = f.begv[grp + 1];
  const int cnt = te0 - tb0;
  const int chunk = (cnt + f.ksplit - 1) / f.ksplit;
  const int tb = tb0 + z * chunk;
  const int te = tb + chunk < te0 ? tb + chunk : te0;
  const long Lrow = (long)f.Rl * f.q, Xrow = (long)f.n * f.s, Rrow = (long)f.Rr * f.s;
  // the term metadata and the skip flag are read together, before any tile load
  int mc, me;
  double mv;
  term_prefetch(f, f.tc, tb, te, lane, mc, me, mv);
  if (f.skip && *f.skip) return;
  // x at this thread's output positions for the dot epilogue, read with the first term
  // (out-of-range positions read element 0 and are not added)
  double xd[4] = {0.0, 0.0, 0.0, 0.0};
  if (f.dots) {
#pragma unroll
    for (int qq = 0; qq < 4; ++qq) {
      const int row = wm * 16 + acc_row<P>(qq, lk), col = wn * 16 + lrow;
      const bool in = row < f.p && col < f.t;
      xd[qq] = f.x[in ? ((long)row * f.n + grp) * f.s + col : 0];
    }
  }
  // thread -> 4 elements of each 32 x 32 tile: r = idx / 32, c = idx % 32, idx = tid + 256 j
  double la[4], xb[4], rb[4], vcur = 0.0;
  auto load = [&](int t, double (&l)[4], double (&x)[4], double (&rr)[4], double& v) {
    int code, e;
    term_get(f, f.tc, t, tb, mc, me, mv, code, e, v);
    const double* Lb = f.L + (long)(code >> 4) * f.q;
    const double* Xi = f.x + (long)(code & 15) * f.s;
    const double* Re = f.Rt + (long)e * f.s;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int idx = tid + 256 * j, r = idx / 32, c = idx % 32;
      l[j] = (r < f.p && c < f.q) ? Lb[r * Lrow + c] : 0.0;
      x[j] = (r < f.q && c < f.s) ? Xi[r * Xrow + c] : 0.0;
      rr[j] = (r < f.t && c < f.s) ? Re[r * Rrow + c] : 0.0;
    }
  };
  if (tb < te) load(tb, la, xb, rb, vcur);
  Acc acc = {0, 0, 0, 0};
  for (int t = tb; t < te; ++t) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int idx = tid + 256 * j, r = idx / 32, c = idx % 32;
      sA[c][r] = (T)la[j];  // A = L rows (m = r) x q (k = c)
      sB[r][c] = (T)xb[j];  // B = x (k = r) x s (n = c)
      sR[c][r] = (T)rb[j];  // B' = Rt^T: k = s (c), n = t (r)
    }
    const double v = vcur;
    if (t + 1 < te) load(t + 1, la, xb, rb, vcur);
    __syncthreads();
    Acc tacc = {0, 0, 0, 0};
    mfma_k32<P>(sA, sB, wm * 16, wn * 16, lk, lrow, tacc);
#pragma unroll
    for (int qq = 0; qq < 4; ++qq) sT[wn * 16 + lrow][wm * 16 + acc_row<P>(qq, lk)] = (T)(v * (double)tacc[qq]);
    __syncthreads();
    mfma_k32<P>(sT, sR, wm * 16, wn * 16, lk, lrow, acc);
    __syncthreads();
  }
  double* Pt = f.partial + ((long)z * f.n + grp) * 1024;
#pragma unroll
  for (int qq = 0; qq < 4; ++qq) Pt[(wm * 16 + acc_row<P>(qq, lk)) * 32 + wn * 16 + lrow] = (double)acc[qq];
  if (f.dots) {
    double d = 0.0;
#pragma unroll
    for (int qq = 0; qq < 4; ++qq) {
      const int row = wm * 16 + acc_row<P>(qq, lk), col = wn * 16 + lrow;
      if (row < f.p && col < f.t) d += (double)acc[qq] * xd[qq];
    }
    store_block_dot(d, f.dots + (long)z * f.n + grp);
  }
}

template <int P>
__global__ __launch_bounds__(256) void fused_apply32_kernel(FusedArgs f) {
  fused_apply32_body<P>(f, blockIdx.y, blockIdx.z);
}

// Ranks above 64: the apply in two stages.
// Stage 1 (slot_product_kernel): S[slot] = L_b x_i for every slot (b, i) of the core,
// p x s, stored in the operand type with rows and columns padded to multiples of 64
// (the padding is written as zeros).  Each product is formed once, where the one-pass
// kernels form it once per term that uses the slot.
// Stage 2 (slot_apply_kernel): per output mode i', 64 x 64 output tiles,
//   part[z][i'][tile32][32 x 32] = sum over the split's terms (slot, e, v) of
//                                  v S[slot] Rt_e^T,
// each term's product accumulated on MFMA (in the accumulate type) and added with its
// coefficient into FP64 accumulators.  The partial tiles have the layout of the
// one-pass kernels (32 x 32 tiles), so the CG reduction sums them unchanged.
constexpr int kStageTile = 64;

inline int pad64(int x) { return (x + kStageTile - 1) / kStageTile * kStageTile; }

template <int P>
__global__ __launch_bounds__(256) void slot_product_kernel(FusedArgs f) {
  using T = typename Prec<P>::T;
  using Acc = typename Prec<P>::Acc;
  if (f.skip && *f.skip) return;
  __shared__ T sA[32][65];
  __shared__ T sB[32][65];
  const int slot = blockIdx.y;
  const int p64 = (f.p + 63) / 64 * 64, s64 = (f.s + 63) / 64 * 64;
  const int tn = s64 / 64;
  const int m0 = (blockIdx.x / tn) * 64, n0 = (blockIdx.x % tn) * 64;
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int wm = wave / 2, wn = wave % 2;
  const int lrow = lane % 16, lk = lane / 16;
  const long Lrow = (long)f.Rl * f.q, Xrow = (long)f.n * f.s;
  const double* Lb = f.L + (long)f.slot_b[slot] * f.q;
  const double* Xi = f.x + (long)f.slot_i[slot] * f.s;
  // A: 64 rows x 32 k (k contiguous in memory); B: 32 k x 64 columns (columns contiguous)
  double ra[8], rb[8];
  auto load = [&](int k0) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int idx = tid + 256 * j;
      const int r = idx / 32, k = idx % 32;
      ra[j] = (m0 + r < f.p && k0 + k < f.q) ? Lb[(m0 + r) * Lrow + k0 + k] : 0.0;
      const int kb = idx / 64, c = idx % 64;
      rb[j] = (k0 + kb < f.q && n0 + c < f.s) ? Xi[(k0 + kb) * Xrow + n0 + c] : 0.0;
    }
  };
  Acc acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = Acc{0, 0, 0, 0};
  const int nks = (f.q + 31) / 32;
  load(0);
  for (int ks = 0; ks < nks; ++ks) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int idx = tid + 256 * j;
      sA[idx % 32][idx / 32] = (T)ra[j];
      sB[idx / 64][idx % 64] = (T)rb[j];
    }
    if (ks + 1 < nks) load((ks + 1) * 32);
    __syncthreads();
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int ni = 0; ni < 2; ++ni)
        mfma_k32o<P, 65>(sA, sB, 0, wm * 32 + mi * 16, wn * 32 + ni * 16, lk, lrow, acc[mi][ni]);
    __syncthreads();
  }
  T* S = static_cast<T*>(f.stage) + ((long)slot * p64 + m0) * s64 + n0;
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int qq = 0; qq < 4; ++qq)
        S[(long)(wm * 32 + mi * 16 + acc_row<P>(qq, lk)) * s64 + wn * 32 + ni * 16 + lrow] = (T)acc[mi][ni][qq];
}

template <int P>
__global__ __launch_bounds__(256) void slot_apply_kernel(FusedArgs f) {
  using T = typename Prec<P>::T;
  using Acc = typename Prec<P>::Acc;
  __shared__ T sA[32][65];
  __shared__ T sB[32][65];
  const int grp = blockIdx.y, z = blockIdx.z;
  const int p64 = (f.p + 63) / 64 * 64, s64 = (f.s + 63) / 64 * 64;
  const int tn = (f.t + 63) / 64;
  const int bm = blockIdx.x / tn, bn = blockIdx.x % tn;
  const int m0 = bm * 64, n0 = bn * 64;
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int wm = wave / 2, wn = wave % 2;
  const int lrow = lane % 16, lk = lane / 16;
  const int tb0 = f.begv[grp], te0 = f.begv[grp + 1];
  const int cnt = te0 - tb0;
  const int chunk = (cnt + f.ksplit - 1) / f.ksplit;
  const int tb = tb0 + z * chunk;
  const int te = tb + chunk < te0 ? tb + chunk : te0;
  const long Rrow = (long)f.Rr * f.s;
  const T* S = static_cast<const T*>(f.stage);
  // the term metadata (slot, e, v) and the skip flag are read together, before any tile
  int ms, me;
  double mv;
  term_prefetch(f, f.ta, tb, te, lane, ms, me, mv);
  if (f.skip && *f.skip) return;
  const int nks = (f.s + 31) / 32;
  // item = (term, k step); A = S[slot] rows m0.., k (in bounds: padded); B = Rt_e^T
  T ra[8];
  double rb[8];
  auto load = [&](int t, int k0) {
    int slot, e;
    double v;
    term_get(f, f.ta, t, tb, ms, me, mv, slot, e, v);
    const T* Sa = S + ((long)slot * p64 + m0) * s64 + k0;
    const double* Re = f.Rt + (long)e * f.s + k0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int idx = tid + 256 * j;
      const int r = idx / 32, k = idx % 32;
      ra[j] = Sa[(long)r * s64 + k];
      rb[j] = (n0 + r < f.t && k0 + k < f.s) ? Re[(n0 + r) * Rrow + k] : 0.0;
    }
  };
  double acc[2][2][4];
  Acc tacc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      tacc[i][j] = Acc{0, 0, 0, 0};
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[i][j][q] = 0.0;
    }
  const long items = (long)(te > tb ? te - tb : 0) * nks;
  if (items > 0) load(tb, 0);
  for (long it = 0; it < items; ++it) {
    const int t = tb + (int)(it / nks), ks = (int)(it % nks);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int idx = tid + 256 * j;
      sA[idx % 32][idx / 32] = ra[j];
      sB[idx % 32][idx / 32] = (T)rb[j];
    }
    if (it + 1 < items) load(tb + (int)((it + 1) / nks), (int)((it + 1) % nks) * 32);
    __syncthreads();
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int ni = 0; ni < 2; ++ni)
        mfma_k32o<P, 65>(sA, sB, 0, wm * 32 + mi * 16, wn * 32 + ni * 16, lk, lrow, tacc[mi][ni]);
    __syncthreads();
    if (ks == nks - 1) {
      int slot, e;
      double v;
      term_get(f, f.ta, t, tb, ms, me, mv, slot, e, v);
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni) {
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[mi][ni][q] += v * (double)tacc[mi][ni][q];
          tacc[mi][ni] = Acc{0, 0, 0, 0};
        }
    }
  }
  // the wave's 32 x 32 quadrant is 32-tile (2 bm + wm, 2 bn + wn), when it exists
  const int rt = 2 * bm + wm, ct = 2 * bn + wn;
  if (rt * 32 < f.p && ct * 32 < f.t) {
    double* Pt = f.partial + (((long)z * f.n + grp) * f.ntiles + rt * f.tiles_n + ct) * 1024;
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int ni = 0; ni < 2; ++ni)
#pragma unroll
        for (int qq = 0; qq < 4; ++qq)
          Pt[(mi * 16 + acc_row<P>(qq, lk)) * 32 + ni * 16 + lrow] = acc[mi][ni][qq];
  }
  if (f.dots) {
    // as in the one-pass kernels: the x loads issued together, then summed in order
    double xv[2][2][4];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int ni = 0; ni < 2; ++ni)
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
          const int row = m0 + wm * 32 + mi * 16 + acc_row<P>(qq, lk), col = n0 + wn * 32 + ni * 16 + lrow;
          const bool in = row < f.p && col < f.t;
          xv[mi][ni][qq] = f.x[in ? ((long)row * f.n + grp) * f.s + col : 0];
        }
    double d = 0.0;
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int ni = 0; ni < 2; ++ni)
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
          const int row = m0 + wm * 32 + mi * 16 + acc_row<P>(qq, lk), col = n0 + wn * 32 + ni * 16 + lrow;
          if (row < f.p && col < f.t) d += acc[mi][ni][qq] * xv[mi][ni][qq];
        }
    store_block_dot(d, f.dots + ((long)z * f.n + grp) * (((f.p + 63) / 64) * tn) + blockIdx.x);
  }
}

size_t fused_stage_elems(const FusedArgs& f) { return (size_t)f.nslot * pad64(f.p) * pad64(f.s); }

// Shared launch of the fused apply of several requests (same mode count n): grid z
// runs over the requests' split ranges zoff[r] .. zoff[r + 1]; every block does
// exactly what the single-request launch does for its (request, mode, tile, split).
template <int P>
__global__ __launch_bounds__(256) void fused_apply32_batch_kernel(FusedBatch b) {
  const int z = blockIdx.z;
  int r = 0;
  while (r + 1 < b.nreq && z >= b.zoff[r + 1]) ++r;
  const FusedArgs& f = b.args[r];
  fused_apply32_body<P>(f, blockIdx.y, z - b.zoff[r]);
}

template <int P>
__global__ __launch_bounds__(256) FUSED2_OCC void fused_apply64_batch_kernel(FusedBatch b) {
  const int z = blockIdx.z;
  int r = 0;
  while (r + 1 < b.nreq && z >= b.zoff[r + 1]) ++r;
  const FusedArgs& f = b.args[r];
  fused_apply64_body<P>(f, blockIdx.y, z - b.zoff[r]);
}

template <int P, int BPW>
__global__ __launch_bounds__(256) FUSED2_OCC void fused_apply16_batch_kernel(FusedBatch b) {
  const int z = blockIdx.z;
  int r = 0;
  while (r + 1 < b.nreq && z >= b.zoff[r + 1]) ++r;
  const FusedArgs& f = b.args[r];
  fused_apply16_body<P, BPW>(f, blockIdx.y, z - b.zoff[r]);
}

int fused_kind(const FusedArgs& f) {
  const int m = std::max(std::max(f.p, f.q), std::max(f.s, f.t));
  return m <= 32 ? FUSED_32 : (m <= 64 ? FUSED_64 : FUSED_TILED);
}

int fused_dot_count(const FusedArgs& f) {
  const int per = fused_kind(f) == FUSED_TILED ? ((f.p + 63) / 64) * ((f.t + 63) / 64) : 1;
  return f.ksplit * f.n * per;
}

int fused_apply_splits(const FusedArgs& f, int max_terms, size_t cap_doubles) {
  const int n = f.n;
  const int ntiles = ((f.p + 31) / 32) * ((f.t + 31) / 32);
  // workgroups per split: the 32 / 64 kernels cover all output tiles of a mode in one
  // and are bound by the latency of their term loop, so they are split down to about one
  // term per workgroup (one workgroup per compute unit); the two-stage kernel has 64 x 64
  // output tiles and far more work per term, and keeps at least two terms per workgroup
  // (about two workgroups per compute unit)
  const bool staged = fused_kind(f) == FUSED_TILED;
  const long per_split = staged ? (long)n * ((f.p + 63) / 64) * ((f.t + 63) / 64) : n;
  const long target = staged ? 512 : 256;
  long ks = (target + per_split - 1) / per_split;
  ks = std::min<long>(ks, std::max(1, staged ? max_terms / 2 : max_terms));
  const long fit = (long)(cap_doubles / ((size_t)n * ntiles * 1024));
  if (fit < 1) throw Error(TNFEM_EINVAL, "fused apply: partial buffer too small");
  ks = std::min<long>(ks, fit);
  return (int)std::max<long>(ks, 1);
}

static hipEvent_t* prof_begin(hipStream_t s);
static void prof_end(hipEvent_t* pair, double flops, hipStream_t s, int kind);

template <int P>
static void launch_fused_kind(const FusedArgs& f, int kind, hipEvent_t* ev, hipStream_t s) {
  const dim3 g1(1, f.n, f.ksplit);
  if (f.n < 1 || f.n > FUSED_MAX_MODES || f.begv[f.n] <= 0 || (kind != FUSED_TILED && !f.tc))
    throw Error(TNFEM_EINVAL, "fused apply: term lists not set or more than 8 modes");
  if (kind == FUSED_32) {
    TN_LAUNCH(ev, fused_apply32_kernel<P>, g1, dim3(256), 0, s, f);
  } else if (kind == FUSED_64) {
    const int bpw = P == 2 ? 4 : fused16_bpw(f);
    if (bpw <= 1) TN_LAUNCH(ev, (fused_apply16_kernel<P == 2 ? 0 : P, 1>), g1, dim3(256), 0, s, f);
    else if (bpw == 2) TN_LAUNCH(ev, (fused_apply16_kernel<P == 2 ? 0 : P, 2>), g1, dim3(256), 0, s, f);
    else TN_LAUNCH(ev, fused_apply64_kernel<P>, g1, dim3(256), 0, s, f);
  } else {
    if (!f.stage || f.nslot <= 0 || fused_stage_elems(f) * sizeof(double) > f.stage_bytes)
      throw Error(TNFEM_EINVAL, "fused apply: stage buffer missing or too small for ranks above 64");
    const dim3 g_prod((pad64(f.p) / 64) * (pad64(f.s) / 64), f.nslot);
    const dim3 g_app(((f.p + 63) / 64) * ((f.t + 63) / 64), f.n, f.ksplit);
    // the profile pair brackets both stages: start at the first dispatch, end at the second
    if (ev) {
      hipExtLaunchKernelGGL(slot_product_kernel<P>, g_prod, dim3(256), 0, s, ev[0], nullptr, 0, f);
      hipExtLaunchKernelGGL(slot_apply_kernel<P>, g_app, dim3(256), 0, s, nullptr, ev[1], 0, f);
    } else {
      hipLaunchKernelGGL(slot_product_kernel<P>, g_prod, dim3(256), 0, s, f);
      hipLaunchKernelGGL(slot_apply_kernel<P>, g_app, dim3(256), 0, s, f);
    }
  }
}

void launch_fused_apply(FusedArgs f, double flops, hipStream_t s, int precision) {
  fused_prepare(f);
  hipEvent_t* ev = prof_begin(s);
  const int kind = fused_kind(f);
  if (precision == 1) launch_fused_kind<1>(f, kind, ev, s);
  else if (precision == 2) launch_fused_kind<2>(f, kind, ev, s);
  else launch_fused_kind<0>(f, kind, ev, s);
  prof_end(ev, flops, s, precision ? PROF_FUSED_LOW : PROF_FUSED);
  TN_CHECK_LAUNCH();
}

void fused_prepare(FusedArgs& f) {
  f.tiles_n = (f.t + 31) / 32;
  f.ntiles = ((f.p + 31) / 32) * f.tiles_n;
}

template <int P>
static void launch_fused_batch_kind(const FusedBatch& b, int n, int kind, hipStream_t s) {
  const int zt = b.zoff[b.nreq];
  const dim3 g1(1, n, zt);
  if (kind == FUSED_32) {
    hipLaunchKernelGGL(fused_apply32_batch_kernel<P>, g1, dim3(256), 0, s, b);
  } else if (kind == FUSED_64) {
    // the requests' block counts differ; the largest sets the slots per wave (a block's
    // result does not depend on it)
    const int bpw = P == 2 ? 4 : b.bpw;
    if (bpw <= 1) hipLaunchKernelGGL((fused_apply16_batch_kernel<P == 2 ? 0 : P, 1>), g1, dim3(256), 0, s, b);
    else if (bpw == 2) hipLaunchKernelGGL((fused_apply16_batch_kernel<P == 2 ? 0 : P, 2>), g1, dim3(256), 0, s, b);
    else hipLaunchKernelGGL(fused_apply64_batch_kernel<P>, g1, dim3(256), 0, s, b);
  } else {
    throw Error(TNFEM_EINVAL, "fused apply batch: ranks above 64 are launched per request");
  }
}

void launch_fused_apply_batch(const FusedBatch& b, int n, int kind, hipStream_t s, int precision) {
  if (b.nreq <= 0) return;
  if (b.nreq > FB_MAX) throw Error(TNFEM_EINVAL, "fused apply batch: too many requests");
  if (precision == 1) launch_fused_batch_kind<1>(b, n, kind, s);
  else if (precision == 2) launch_fused_batch_kind<2>(b, n, kind, s);
  else launch_fused_batch_kind<0>(b, n, kind, s);
  TN_CHECK_LAUNCH();
}

static int blocks_for(long total);

// Sum over the ksplit split partials src[z * stride], z = 0 .. ksplit - 1, in split order.
// The first 32 loads are issued together (indices clamped, so every load is in bounds;
// the clamped copies are not added), then summed in order.
__device__ inline double sum_splits(const double* src, long stride, int ksplit) {
  constexpr int U = 32;
  if (ksplit <= 0) return 0.0;
  double v[U];
#pragma unroll
  for (int u = 0; u < U; ++u) v[u] = src[(long)(u < ksplit ? u : ksplit - 1) * stride];
  double w = 0.0;
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (u < ksplit) w += v[u];
  for (int z = U; z < ksplit; ++z) w += src[(long)z * stride];
  return w;
}

// y[row][grp][col] = sum over splits of the fused partial tiles (split order), or
// g[e] minus that sum when g is given (g may be y).
__global__ void fused_sum_kernel(FusedArgs f, double* y, const double* g) {
  if (f.skip && *f.skip) return;
  const long N = (long)f.p * f.n * f.t;
  const long stride = (long)f.n * f.ntiles * 1024;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < N; e += (long)gridDim.x * blockDim.x) {
    const int col = e % f.t, grp = (e / f.t) % f.n, row = e / ((long)f.t * f.n);
    const int tile = (row / 32) * f.tiles_n + col / 32;
    const double* src = f.partial + ((long)grp * f.ntiles + tile) * 1024 + (row % 32) * 32 + (col % 32);
    const double v = sum_splits(src, stride, f.ksplit);
    y[e] = g ? g[e] - v : v;
  }
}

// The same for two applies at once (their partials in separate buffers): elements
// 0 .. N1 - 1 of the grid belong to the first, the rest to the second.
__global__ void fused_sum2_kernel(FusedArgs f1, double* y1, const double* g1, FusedArgs f2, double* y2,
                                  const double* g2) {
  const long N1 = (long)f1.p * f1.n * f1.t, N2 = (long)f2.p * f2.n * f2.t;
  for (long e0 = blockIdx.x * (long)blockDim.x + threadIdx.x; e0 < N1 + N2; e0 += (long)gridDim.x * blockDim.x) {
    const bool first = e0 < N1;
    const FusedArgs& f = first ? f1 : f2;
    const long e = first ? e0 : e0 - N1;
    const long stride = (long)f.n * f.ntiles * 1024;
    const int col = e % f.t, grp = (e / f.t) % f.n, row = e / ((long)f.t * f.n);
    const int tile = (row / 32) * f.tiles_n + col / 32;
    const double* src = f.partial + ((long)grp * f.ntiles + tile) * 1024 + (row % 32) * 32 + (col % 32);
    const double v = sum_splits(src, stride, f.ksplit);
    const double* g = first ? g1 : g2;
    double* y = first ? y1 : y2;
    y[e] = g ? g[e] - v : v;
  }
}

void launch_fused_sum2(FusedArgs f1, double* y1, const double* g1, FusedArgs f2, double* y2, const double* g2,
                       hipStream_t s) {
  if (f1.skip || f2.skip) throw Error(TNFEM_EINVAL, "fused sum of two applies: no stop flag");
  f1.tiles_n = (f1.t + 31) / 32;
  f1.ntiles = ((f1.p + 31) / 32) * f1.tiles_n;
  f2.tiles_n = (f2.t + 31) / 32;
  f2.ntiles = ((f2.p + 31) / 32) * f2.tiles_n;
  const long N = (long)f1.p * f1.n * f1.t + (long)f2.p * f2.n * f2.t;
  const int nb = (int)std::min<long>(std::max<long>((N + 63) / 64, 1), 4096);
  hipLaunchKernelGGL(fused_sum2_kernel, dim3(nb), dim3(64), 0, s, f1, y1, g1, f2, y2, g2);
  TN_CHECK_LAUNCH();
}

void launch_fused_sum(FusedArgs f, double* y, hipStream_t s, const double* minus_from) {
  f.tiles_n = (f.t + 31) / 32;
  f.ntiles = ((f.p + 31) / 32) * f.tiles_n;
  const long N = (long)f.p * f.n * f.t;
  // 64-thread blocks: the split sums of a local vector spread over more compute units
  const int nb = (int)std::min<long>(std::max<long>((N + 63) / 64, 1), 4096);
  hipLaunchKernelGGL(fused_sum_kernel, dim3(nb), dim3(64), 0, s, f, y, minus_from);
  TN_CHECK_LAUNCH();
}

// ----------------------------------------------------------------------------- CG iteration kernels
// Block partials: parts[PART_RZ + (k % 2) * CG_MAXB + blk] etc.; scalars scal[CG_RZ0 + k % 2].

constexpr int PART_RZ = 0, PART_RR = 2 * CG_MAXB, PART_PQ = 4 * CG_MAXB;
// cg_step reuses the p.q region (and the one after it) for the apply's (z, B z) partials
static_assert(CG_DOT_OFFSET == PART_PQ && CG_DOT_MAX == 2 * CG_MAXB, "dot partial region");

// z_j = sum_i brow[i] r_i over the bn lanes of a block (aligned groups of bnp lanes);
// every lane of the group takes part in the exchanges.
__device__ inline double block_apply(const double* brow, double ri, int bn, int gbase, bool act) {
  double zi = 0.0;
  if (bn <= 8) {
    // rows of up to 8 entries: all loads issued before the first product
    double b[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) b[i] = (act && i < bn) ? brow[i] : 0.0;
#pragma unroll
    for (int i = 0; i < 8; ++i)
      if (i < bn) {
        const double rv = __shfl(ri, gbase + i, 64);
        if (act) zi += b[i] * rv;
      }
    return zi;
  }
  for (int i = 0; i < bn; ++i) {
    const double rv = __shfl(ri, gbase + i, 64);
    if (act) zi += brow[i] * rv;
  }
  return zi;
}

__device__ inline double sum_parts(const double* a, int nb) {
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += a[b];
  return s;
}

// w = sum of split partials (or w given directly); p = z + beta p; q = w + beta q; block partials of p.q.
// First checks convergence of iteration k from the update's partials.
__device__ __forceinline__ void cg_reduce_dir_body(const CgIterArgs& a, const int k, const int bid) {
  __shared__ double red[4];
  if (a.flag[CG_DONE]) return;
  const int nb = a.nb_upd;
  const int par = k & 1;
  const double rr = sum_parts(a.parts + PART_RR + par * CG_MAXB, nb);
  if (rr <= a.scal[CG_THR2] || k >= a.maxit) {
    if (bid == 0 && threadIdx.x == 0) {
      a.flag[CG_DONE] = 1;
      a.flag[CG_ITERS] = k;
    }
    return;
  }
  const double rz = sum_parts(a.parts + PART_RZ + par * CG_MAXB, nb);
  const double beta = (k == 0) ? 0.0 : rz / a.scal[CG_RZ0 + (par ^ 1)];
  if (bid == 0 && threadIdx.x == 0) {
    a.scal[CG_RZ0 + par] = rz;
    a.flag[CG_ITERS] = k;
  }
  double loc = 0.0;
  for (int e = bid * 256 + threadIdx.x; e < a.N; e += a.nb_dir * 256) {
    double w;
    if (a.ksplit > 0) {
      // e = (row * n + grp) * t + col
      const int col = e % a.t, grp = (e / a.t) % a.n, row = e / (a.t * a.n);
      const int tile = (row / 32) * a.tiles_n + col / 32;
      const long stride = (long)a.n * a.ntiles * 1024;
      const double* src = a.partial + ((long)grp * a.ntiles + tile) * 1024 + (row % 32) * 32 + (col % 32);
      w = sum_splits(src, stride, a.ksplit);
    } else {
      w = a.w[e];
    }
    const double pi = a.z[e] + beta * a.p[e];
    const double qi = w + beta * a.q[e];
    a.p[e] = pi;
    a.q[e] = qi;
    loc += pi * qi;
  }
  const double tot = block_sum<256>(loc, red);
  if (threadIdx.x == 0) a.parts[PART_PQ + bid] = tot;
}

__global__ __launch_bounds__(256) void cg_reduce_dir_kernel(CgIterArgs a, int k) { cg_reduce_dir_body(a, k, blockIdx.x); }


// x += alpha p; r -= alpha q; z = M^-1 r; block partials of r.z and r.r for iteration k + 1.
__device__ __forceinline__ void cg_update2_body(const CgIterArgs& a, const int k, const int bid) {
  __shared__ double red[4];
  if (a.flag[CG_DONE]) return;
  const int nb = a.nb_upd;
  const double pq = sum_parts(a.parts + PART_PQ, a.nb_dir);
  if (!(pq > 0.0)) {  // breakdown: stop without updating
    if (bid == 0 && threadIdx.x == 0) {
      a.flag[CG_DONE] = 2;
      a.flag[CG_ITERS] = k;
    }
    return;
  }
  const double alpha = a.scal[CG_RZ0 + (k & 1)] / pq;
  double lrz = 0.0, lrr = 0.0;
  const int bn = a.bn, bnp = a.bnp, t = a.bt;
  const long total = (long)(a.N / bn) * bnp;
  const int gbase = (threadIdx.x % 64) & ~(bnp - 1);
  for (long idx = bid * 256 + threadIdx.x; idx < total; idx += (long)nb * 256) {
    const int j = (int)(idx % bnp);
    const long blk = idx / bnp;
    const bool act = j < bn;
    const long e = ((blk / t) * bn + j) * t + blk % t;
    double ri = 0.0;
    if (act) {
      a.x[e] += alpha * a.p[e];
      ri = a.r[e] - alpha * a.q[e];
      a.r[e] = ri;
    }
    const double zi = block_apply(a.binv + blk * bn * bn + (long)j * bn, ri, bn, gbase, act);
    if (act) {
      a.z[e] = zi;
      lrz += ri * zi;
      lrr += ri * ri;
    }
  }
  const double trz = block_sum<256>(lrz, red);
  const double trr = block_sum<256>(lrr, red);
  const int par = (k + 1) & 1;
  if (threadIdx.x == 0) {
    a.parts[PART_RZ + par * CG_MAXB + bid] = trz;
    a.parts[PART_RR + par * CG_MAXB + bid] = trr;
  }
}

__global__ __launch_bounds__(256) void cg_update2_kernel(CgIterArgs a, int k) { cg_update2_body(a, k, blockIdx.x); }

// One iteration of the same preconditioned CG in the Chronopoulos-Gear arrangement,
// after the fused apply of z_k that also wrote the partials of delta = (z_k, B z_k):
//   gamma = (r_k, z_k); beta = gamma / gamma_{k-1}; (p_k, B p_k) = delta - beta gamma / alpha_{k-1}
//   (delta alone at k = 0, beta = 0); alpha = gamma / (p_k, B p_k);
//   p = z + beta p; q = w + beta q (q = B p); x += alpha p; r -= alpha q; z = M^-1 r;
//   block partials of (r, z), (r, r) for iteration k + 1.
// Convergence of iteration k is tested first, from the previous step's partials.
template <int NT>
__device__ __forceinline__ void cg_step_body(const CgIterArgs& a, const int k, const int bid) {
  __shared__ double red[NT / 64];
  constexpr int U = 32;    // split partials read with the vectors (the rest after them)
  constexpr int BPRE = 8;  // preconditioner rows of up to 8 entries are read with the vectors
  const int nb_read = k == 0 ? a.nb_upd : a.nb_step;  // partials of the previous kernel
  const int nb = a.nb_step;
  const int par = k & 1;
  const int lane = threadIdx.x % 64;
  // element layout [p][n][t]: the preconditioner block (a, c) holds the n entries of mode
  // index j (n = bn, t = bt, checked on the host); 32-bit index arithmetic (N < 2^28)
  const unsigned bn = a.bn, t = a.bt, bnp = a.bnp, lbnp = __builtin_ctz(a.bnp);
  const int total = (a.N / a.bn) * a.bnp;
  const int gbase = lane & ~(a.bnp - 1);
  const long stride = (long)a.n * a.ntiles * 1024;
  const int ks = a.ksplit;
  const bool bpre = bn <= BPRE;
  struct Elem {
    unsigned e;
    bool act;
    double z, p, q, x, r;
    double w[U];
    double b[BPRE];
    const double* brow;
    const double* src;
  };
  const __amdgpu_buffer_rsrc_t rpart = tile_rsrc(a.partial, (long)(ks > 0 ? ks : 1) * stride);
  const __amdgpu_buffer_rsrc_t rz = tile_rsrc(a.z, a.N), rpv = tile_rsrc(a.p, a.N), rq = tile_rsrc(a.q, a.N),
                               rx = tile_rsrc(a.x, a.N), rrv = tile_rsrc(a.r, a.N);
  auto load = [&](int idx, Elem& el) {
    const unsigned j = (unsigned)idx & (bnp - 1), blk = (unsigned)idx >> lbnp;
    const unsigned row = blk / t, col = blk - row * t;
    el.act = idx < total && j < bn;
    el.e = (row * bn + j) * t + col;
    el.brow = a.binv + (long)blk * bn * bn + j * bn;
    const int tile = (int)(row / 32) * a.tiles_n + (int)(col / 32);
    el.src = a.partial + ((long)j * a.ntiles + tile) * 1024 + (row % 32) * 32 + (col % 32);
    el.z = el.p = el.q = el.x = el.r = 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) el.w[u] = 0.0;
    if (el.act) {
      // buffer loads: one offset register for the split partials (the split step in the
      // scalar offset) and one for the five vectors
      const int vo = (int)(el.src - a.partial) * 8, ve = (int)el.e * 8;
#pragma unroll
      for (int u = 0; u < U; ++u) el.w[u] = tile_load(rpart, vo, (int)((u < ks ? u : ks - 1) * stride * 8));
      el.z = tile_load(rz, ve, 0);
      el.p = tile_load(rpv, ve, 0);
      el.q = tile_load(rq, ve, 0);
      el.x = tile_load(rx, ve, 0);
      el.r = tile_load(rrv, ve, 0);
    }
#pragma unroll
    for (int i = 0; i < BPRE; ++i) el.b[i] = (bpre && el.act && i < (int)bn) ? el.brow[i] : 0.0;
  };
  // B z at the element: the ordered sum over the splits
  auto bz = [&](const Elem& el) {
    double w = 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (u < ks) w += el.w[u];
    for (int z = U; z < ks; ++z) w += el.src[(long)z * stride];
    return w;
  };
  // everything the first element needs is read together with the done flag and the
  // partial sums; the decisions below wait for all of it at once
  const int idx0 = bid * NT + threadIdx.x;
  Elem cur;
  load(idx0, cur);
  const int done = a.flag[CG_DONE];
  const double thr2 = a.scal[CG_THR2];
  const double rz_prev = a.scal[CG_RZ0 + (par ^ 1)], alpha_prev = a.scal[CG_ALPHA0 + (par ^ 1)];
  // the three partial sums, lane-strided and then a fixed-order wavefront sum: every
  // wavefront forms the same values
  const double* prr = a.parts + PART_RR + par * CG_MAXB;
  const double* prz = a.parts + PART_RZ + par * CG_MAXB;
  const double* pd = a.parts + CG_DOT_OFFSET;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll 4
  for (int i = lane; i < nb_read; i += 64) {
    s0 += prr[i];
    s1 += prz[i];
  }
#pragma unroll 4
  for (int i = lane; i < a.ndots; i += 64) s2 += pd[i];
  if (done) return;
  const double rr = wave_sum(s0);
  if (rr <= thr2 || k >= a.maxit) {
    if (bid == 0 && threadIdx.x == 0) {
      a.flag[CG_DONE] = 1;
      a.flag[CG_ITERS] = k;
    }
    return;
  }
  const double gamma = wave_sum(s1);
  const double delta = wave_sum(s2);
  double beta = 0.0, pq = delta;
  if (k > 0) {
    beta = gamma / rz_prev;
    pq = delta - beta * gamma / alpha_prev;
  }
  if (!(pq > 0.0)) {  // breakdown: stop without updating
    if (bid == 0 && threadIdx.x == 0) {
      a.flag[CG_DONE] = 2;
      a.flag[CG_ITERS] = k;
    }
    return;
  }
  const double alpha = gamma / pq;
  if (bid == 0 && threadIdx.x == 0) {
    a.scal[CG_RZ0 + par] = gamma;
    a.scal[CG_ALPHA0 + par] = alpha;
    a.flag[CG_ITERS] = k;
  }
  double lrz = 0.0, lrr = 0.0;
  for (int idx = idx0; idx < total; idx += nb * NT) {
    if (idx != idx0) load(idx, cur);
    double ri = 0.0;
    if (cur.act) {
      const unsigned e = cur.e;
      const double pi = cur.z + beta * cur.p;
      const double qi = bz(cur) + beta * cur.q;
      a.p[e] = pi;
      a.q[e] = qi;
      a.x[e] = cur.x + alpha * pi;
      ri = cur.r - alpha * qi;
      a.r[e] = ri;
    }
    double zi = 0.0;
    if (bpre) {
#pragma unroll
      for (int i = 0; i < BPRE; ++i)
        if (i < (int)bn) zi += cur.b[i] * __shfl(ri, gbase + i, 64);
    } else {
      zi = block_apply(cur.brow, ri, bn, gbase, cur.act);
    }
    if (cur.act) {
      a.z[cur.e] = zi;
      lrz += ri * zi;
      lrr += ri * ri;
    }
  }
  const double trz = block_sum<NT>(lrz, red);
  const double trr = block_sum<NT>(lrr, red);
  const int npar = (k + 1) & 1;
  if (threadIdx.x == 0) {
    a.parts[PART_RZ + npar * CG_MAXB + bid] = trz;
    a.parts[PART_RR + npar * CG_MAXB + bid] = trr;
  }
}

template <int NT>
__global__ __launch_bounds__(NT) void cg_step_kernel(CgIterArgs a, int k) {
  cg_step_body<NT>(a, k, blockIdx.x);
}

// r = g - Bx (Bx given, or summed from a fused apply's split partials when bx is null);
// z = M^-1 r; p = q = 0; block partials of r.z, r.r (parity 0);
// the last block also derives res, thr and the skip decision for the host.
__global__ __launch_bounds__(256) void cg_init2_kernel(CgIterArgs a, const double* g, const double* bx, double tol) {
  __shared__ double red[4];
  __shared__ bool am_last;
  double lrz = 0.0, lrr = 0.0, lgg = 0.0;
  const int bn = a.bn, bnp = a.bnp, t = a.bt;
  const long total = (long)(a.N / bn) * bnp;
  const int gbase = (threadIdx.x % 64) & ~(bnp - 1);
  for (long idx = blockIdx.x * 256 + threadIdx.x; idx < total; idx += (long)gridDim.x * 256) {
    const int j = (int)(idx % bnp);
    const long blk = idx / bnp;
    const bool act = j < bn;
    const long e = ((blk / t) * bn + j) * t + blk % t;
    double gi = 0.0, ri = 0.0;
    if (act) {
      gi = g[e];
      double bxe;
      if (bx) {
        bxe = bx[e];
      } else {
        // B x straight from the fused apply's split partial tiles (mode j, row, col)
        const int row = (int)(blk / t), col = (int)(blk % t);
        const int tile = (row / 32) * a.tiles_n + col / 32;
        const double* src = a.partial + ((long)j * a.ntiles + tile) * 1024 + (row % 32) * 32 + (col % 32);
        bxe = sum_splits(src, (long)a.n * a.ntiles * 1024, a.ksplit);
      }
      ri = gi - bxe;
      a.r[e] = ri;
      a.p[e] = 0.0;
      a.q[e] = 0.0;
    }
    const double zi = block_apply(a.binv + blk * bn * bn + (long)j * bn, ri, bn, gbase, act);
    if (act) {
      a.z[e] = zi;
      lrz += ri * zi;
      lrr += ri * ri;
      lgg += gi * gi;
    }
  }
  const double trz = block_sum<256>(lrz, red);
  const double trr = block_sum<256>(lrr, red);
  const double tgg = block_sum<256>(lgg, red);
  if (threadIdx.x == 0) {
    a.parts[PART_RZ + blockIdx.x] = trz;
    a.parts[PART_RR + blockIdx.x] = trr;
    a.parts[PART_PQ + blockIdx.x] = tgg;  // scratch for the gg total
    __threadfence();
    am_last = atomicAdd(&a.flag[CG_COUNTER], 1) == (int)gridDim.x - 1;
  }
  __syncthreads();
  if (!am_last || threadIdx.x != 0) return;
  __threadfence();
  const int nb = gridDim.x;
  const double rr = sum_parts(a.parts + PART_RR, nb), gg = sum_parts(a.parts + PART_PQ, nb);
  const double gn = sqrt(gg);
  const double res = gg > 0.0 ? sqrt(rr) / gn : (rr == 0.0 ? 0.0 : 1.0);
  a.scal[CG_GG] = gg;
  a.scal[CG_RES] = res;
  // beside the flags, so that one copy brings both to the host
  *reinterpret_cast<double*>(a.flag + CG_RES_COPY) = res;
  a.flag[CG_ITERS] = 0;
  if (a.keep_thr) {
    a.flag[CG_DONE] = (rr <= a.scal[CG_THR2] || a.maxit <= 0) ? 1 : 0;
  } else {
    const double thr = fmax(0.1 * res, 0.5 * tol) * gn;
    a.scal[CG_THR2] = thr * thr;
    a.flag[CG_DONE] = (res <= 0.5 * tol || a.maxit <= 0) ? 1 : 0;
  }
  a.flag[CG_COUNTER] = 0;
}

int cg_dir_blocks(int n) {
  int b = (n + 255) / 256;
  return b < 1 ? 1 : (b > CG_MAXB ? CG_MAXB : b);
}

void launch_cg_init2(const CgIterArgs& a, const double* g, const double* bx, double tol, hipStream_t s) {
  if (a.bn < 1 || a.bnp < a.bn || a.bnp > 64 || !a.binv) throw Error(TNFEM_EINVAL, "CG: block preconditioner not set");
  hipLaunchKernelGGL(cg_init2_kernel, dim3(a.nb_upd), dim3(256), 0, s, a, g, bx, tol);
  TN_CHECK_LAUNCH();
}
void launch_cg_reduce_dir(const CgIterArgs& a, int k, hipStream_t s) {
  hipLaunchKernelGGL(cg_reduce_dir_kernel, dim3(a.nb_dir), dim3(256), 0, s, a, k);
  TN_CHECK_LAUNCH();
}
void launch_cg_update2(const CgIterArgs& a, int k, hipStream_t s) {
  hipLaunchKernelGGL(cg_update2_kernel, dim3(a.nb_upd), dim3(256), 0, s, a, k);
  TN_CHECK_LAUNCH();
}
void cg_step_check(const CgIterArgs& a) {
  if (a.ndots <= 0 || a.ndots > CG_DOT_MAX || a.ksplit <= 0) throw Error(TNFEM_EINVAL, "cg_step: needs fused partials");
  if (a.bn != a.n || a.bt != a.t || a.bn < 1 || a.bnp < a.bn || a.bnp > 64 || (a.bnp & (a.bnp - 1)) || !a.binv)
    throw Error(TNFEM_EINVAL, "cg_step: preconditioner blocks must be the mode fibres of the apply output");
  if (a.N < 0 || a.N >= (1 << 28) || a.N % a.bn) throw Error(TNFEM_EINVAL, "cg_step: vector length out of range");
  if ((a.nt_step != 64 && a.nt_step != 256) || a.nb_step < 1 || a.nb_step > CG_MAXB || a.nb_upd < 1 ||
      a.nb_upd > CG_MAXB)
    throw Error(TNFEM_EINVAL, "cg_step: launch shape not set (cg_step_shape)");
}

void cg_step_shape(CgIterArgs& a) {
  if (a.bn < 1 || a.bnp < a.bn) throw Error(TNFEM_EINVAL, "cg_step: block preconditioner not set");
  const long total = (long)(a.N / a.bn) * a.bnp;
  const long b64 = (total + 63) / 64;
  if (b64 <= CG_MAXB) {
    a.nt_step = 64;
    a.nb_step = (int)std::max<long>(b64, 1);
  } else {
    a.nt_step = 256;
    a.nb_step = (int)std::min<long>((total + 255) / 256, CG_MAXB);
  }
}

void launch_cg_step(const CgIterArgs& a, int k, hipStream_t s) {
  cg_step_check(a);
  if (a.nt_step == 64) hipLaunchKernelGGL(cg_step_kernel<64>, dim3(a.nb_step), dim3(64), 0, s, a, k);
  else hipLaunchKernelGGL(cg_step_kernel<256>, dim3(a.nb_step), dim3(256), 0, s, a, k);
  TN_CHECK_LAUNCH();
}

// Shared launches of the CG iteration kernels of several requests: grid x runs over
// the requests' block ranges boff[r] .. boff[r + 1] (nb_dir or nb_upd blocks each).
__device__ inline int cg_batch_request(const CgBatch& b, int x) {
  int r = 0;
  while (r + 1 < b.nreq && x >= b.boff[r + 1]) ++r;
  return r;
}

__global__ __launch_bounds__(256) void cg_reduce_dir_batch_kernel(CgBatch b, int k) {
  const int r = cg_batch_request(b, blockIdx.x);
  const CgIterArgs a = b.args[r];
  cg_reduce_dir_body(a, k, blockIdx.x - b.boff[r]);
}

__global__ __launch_bounds__(256) void cg_update2_batch_kernel(CgBatch b, int k) {
  const int r = cg_batch_request(b, blockIdx.x);
  const CgIterArgs a = b.args[r];
  cg_update2_body(a, k, blockIdx.x - b.boff[r]);
}

template <int NT>
__global__ __launch_bounds__(NT) void cg_step_batch_kernel(CgBatch b, int k) {
  const int r = cg_batch_request(b, blockIdx.x);
  const CgIterArgs a = b.args[r];
  cg_step_body<NT>(a, k, blockIdx.x - b.boff[r]);
}

void launch_cg_reduce_dir_batch(const CgBatch& b, int k, hipStream_t s) {
  if (b.nreq <= 0) return;
  if (b.nreq > FB_MAX) throw Error(TNFEM_EINVAL, "CG batch: too many requests");
  hipLaunchKernelGGL(cg_reduce_dir_batch_kernel, dim3(b.boff[b.nreq]), dim3(256), 0, s, b, k);
  TN_CHECK_LAUNCH();
}

void launch_cg_update2_batch(const CgBatch& b, int k, hipStream_t s) {
  if (b.nreq <= 0) return;
  if (b.nreq > FB_MAX) throw Error(TNFEM_EINVAL, "CG batch: too many requests");
  hipLaunchKernelGGL(cg_update2_batch_kernel, dim3(b.boff[b.nreq]), dim3(256), 0, s, b, k);
  TN_CHECK_LAUNCH();
}

void launch_cg_step_batch(const CgBatch& b, int k, hipStream_t s) {
  if (b.nreq <= 0) return;
  if (b.nreq > FB_MAX) throw Error(TNFEM_EINVAL, "CG batch: too many requests");
  if (b.nt == 64) hipLaunchKernelGGL(cg_step_batch_kernel<64>, dim3(b.boff[b.nreq]), dim3(64), 0, s, b, k);
  else if (b.nt == 256) hipLaunchKernelGGL(cg_step_batch_kernel<256>, dim3(b.boff[b.nreq]), dim3(256), 0, s, b, k);
  else throw Error(TNFEM_EINVAL, "CG batch: step block size must be 64 or 256");
  TN_CHECK_LAUNCH();
}

// ----------------------------------------------------------------------------- explicit local matrix

// Stage 1: M[b][j][i][c][c'] = sum_e A2[(b n + i) n + j][e] Rt[c][e][c']  (A2: dense operator core,
// rows (b, in-index i), columns (out-index j, e)).
__global__ void local_matrix_r_kernel(int Rl, int n, int Rr, int t, const double* A2, const double* Rt, double* M) {
  const long tt = (long)t * t;
  const long total = (long)Rl * n * n * tt;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
    const int c2 = idx % t;
    const int c = (idx / t) % t;
    const long bji = idx / tt;
    const int i = bji % n;
    const int j = (bji / n) % n;
    const int b = bji / ((long)n * n);
    const double* a = A2 + (((long)b * n + i) * n + j) * Rr;
    const double* r = Rt + (long)c * Rr * t + c2;
    double s = 0.0;
    for (int e = 0; e < Rr; ++e) s += a[e] * r[(long)e * t];
    M[idx] = s;
  }
}

// Stage 2: Bm[(a n + j) t + c][(a' n + i) t + c'] = sum_b L[a][b][a'] M[b][j][i][c][c'].
__global__ void local_matrix_l_kernel(int p, int n, int t, int Rl, const double* L, const double* M, double* Bm) {
  const long N = (long)p * n * t;
  const long total = N * N;
  const long tt = (long)t * t, slab = (long)n * n * tt;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
    const long row = idx / N, col = idx % N;
    const int c = row % t, j = (row / t) % n, a = row / ((long)t * n);
    const int c2 = col % t, i = (col / t) % n, a2 = col / ((long)t * n);
    const double* m = M + ((long)j * n + i) * tt + (long)c * t + c2;
    const double* l = L + (long)a * Rl * p + a2;
    double s = 0.0;
    for (int b = 0; b < Rl; ++b) s += l[(long)b * p] * m[b * slab];
    Bm[idx] = s;
  }
}

void launch_local_matrix(int p, int n, int t, int Rl, int Rr, const double* L, const double* A2, const double* Rt,
                         double* M, double* Bm, hipStream_t s) {
  const long m_total = (long)Rl * n * n * t * t;
  const long b_total = (long)p * n * t * (long)p * n * t;
  hipLaunchKernelGGL(local_matrix_r_kernel, dim3(blocks_for(m_total)), dim3(256), 0, s, Rl, n, Rr, t, A2, Rt, M);
  TN_CHECK_LAUNCH();
  hipLaunchKernelGGL(local_matrix_l_kernel, dim3(blocks_for(b_total)), dim3(256), 0, s, p, n, t, Rl, L, M, Bm);
  TN_CHECK_LAUNCH();
}

// y = Bm z, Bm N x N row-major; one wavefront per row, fixed reduction order.
__global__ __launch_bounds__(256) void dense_matvec_kernel(int N, const double* Bm, const double* z, double* y,
                                                           const int* skip) {
  if (skip && *skip) return;
  const int lane = threadIdx.x % 64;
  const long row = (long)blockIdx.x * 4 + threadIdx.x / 64;
  if (row >= N) return;
  const double* b = Bm + row * N;
  double s = 0.0;
  for (int c = lane; c < N; c += 64) s += b[c] * z[c];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) y[row] = s;
}

void launch_dense_matvec(int N, const double* Bm, const double* z, double* y, const int* skip, hipStream_t s) {
  if (N <= 0) return;
  hipLaunchKernelGGL(dense_matvec_kernel, dim3((N + 3) / 4), dim3(256), 0, s, N, Bm, z, y, skip);
  TN_CHECK_LAUNCH();
}

// ----------------------------------------------------------------------------- block-Jacobi preconditioner

constexpr int BLK_MAXN = 8;

// One wavefront per block (a, c); lane = 8 j + i holds entry (j, i) of [m | m^{-1}]
// (modes n < 8 padded with the identity).  The blocks are principal submatrices of
// the SPD local operator, so Gauss-Jordan needs no pivoting; the pivot row and
// column entries are exchanged between lanes at each step.
// The entries of block (a, c) use only the diagonal elements L[a, alpha, a] and
// Rt[c, beta, c] of the interfaces: each wavefront first gathers those (Rl + Rr
// values, a few loads per lane) into LDS, so the term loop reads LDS instead of one
// scattered global load per term and interface (the same sums in the same order).
// The block loop runs the same number of times in every wavefront of a workgroup
// (inactive blocks skip the work), so the LDS staging can use workgroup barriers.
constexpr int BLK_RMAX = 256;  // interface ranks staged in LDS (more: read from memory)

__global__ __launch_bounds__(256) void local_block_inv_kernel(int p, int n, int t, int Rl, int Rr, const double* L,
                                                             const double* Rt, const int* beg, const int* kb,
                                                             const int* ke, const double* kv, double* binv) {
  __shared__ double sL[4][BLK_RMAX], sR[4][BLK_RMAX];
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const long nblk = (long)p * t;
  const int j = lane / BLK_MAXN, i = lane % BLK_MAXN;
  const bool act = j < n && i < n;
  const bool staged = Rl <= BLK_RMAX && Rr <= BLK_RMAX;
  for (long base = (long)blockIdx.x * 4; base < nblk; base += (long)gridDim.x * 4) {
    const long blk = base + wave;
    const bool live = blk < nblk;
    const int a = live ? (int)(blk / t) : 0, c = live ? (int)(blk % t) : 0;
    if (staged) {
      __syncthreads();  // the previous block's reads of sL / sR are done
      if (live) {
        for (int q = lane; q < Rl; q += 64) sL[wave][q] = L[((long)a * Rl + q) * p + a];
        for (int q = lane; q < Rr; q += 64) sR[wave][q] = Rt[((long)c * Rr + q) * t + c];
      }
      __syncthreads();
    }
    if (!live) continue;
    double m = (j == i) ? 1.0 : 0.0;
    if (act) {
      m = 0.0;
      const int pr = j * n + i;
      if (staged) {
        for (int k = beg[pr]; k < beg[pr + 1]; ++k) m += kv[k] * sL[wave][kb[k]] * sR[wave][ke[k]];
      } else {
        for (int k = beg[pr]; k < beg[pr + 1]; ++k)
          m += kv[k] * L[((long)a * Rl + kb[k]) * p + a] * Rt[((long)c * Rr + ke[k]) * t + c];
      }
    }
    double v = (j == i) ? 1.0 : 0.0;
    for (int col = 0; col < n; ++col) {
      const double piv = __shfl(m, col * BLK_MAXN + col, 64);
      const double mrow = __shfl(m, col * BLK_MAXN + i, 64);
      const double vrow = __shfl(v, col * BLK_MAXN + i, 64);
      const double f = __shfl(m, j * BLK_MAXN + col, 64);
      if (j == col) {
        m = mrow / piv;
        v = vrow / piv;
      } else {
        m -= f * (mrow / piv);
        v -= f * (vrow / piv);
      }
    }
    if (act) binv[blk * n * n + (long)j * n + i] = v;
  }
}

void launch_local_block_inv(int p, int n, int t, int Rl, int Rr, const double* L, const double* Rt, const int* beg,
                            const int* kb, const int* ke, const double* kv, double* binv, hipStream_t s) {
  if (n < 1 || n > BLK_MAXN) throw Error(TNFEM_EINVAL, "block preconditioner: mode size out of range");
  const long nblk = (long)p * t;
  if (nblk <= 0) return;
  const unsigned grid = (unsigned)std::min<long>((nblk + 3) / 4, 2048);
  hipLaunchKernelGGL(local_block_inv_kernel, dim3(grid), dim3(256), 0, s, p, n, t, Rl, Rr, L, Rt, beg, kb, ke, kv,
                     binv);
  TN_CHECK_LAUNCH();
}

// ----------------------------------------------------------------------------- QR

constexpr int QR_NT = 1024;
constexpr size_t QR_LDS_BYTES = 160 * 1024 - 2048;  // gfx950: 160 KB of LDS per workgroup

// Householder QR with columns owned by wavefronts (column col belongs to wave
// col % waves) and rows by lanes (row i to lane i % 64) in every phase, so no
// lane reads another lane's writes without a barrier in between.  The owner of
// column j + 1 applies reflector j to it first and forms reflector j + 1 at
// once, so each column costs one barrier; Q is accumulated by every wave for its
// own columns over all reflectors without barriers.
template <bool LDS>
__device__ __forceinline__ void qr_owner_body(int m, int n, const double* A, int lda, double* Q, int ldq, double* R,
                                              int ldr, double* ws, double* dyn) {
  constexpr int NW = QR_NT / 64;
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int c = m < n ? m : n;
  double* base = LDS ? dyn : ws;
  double* W = base;                  // m x n, column-major
  double* Qc = base + (long)m * n;   // m x c, column-major
  double* tau = Qc + (long)m * c;    // c
  double* diag = tau + c;            // c
  for (long idx = tid; idx < (long)m * n; idx += QR_NT) {
    const int i = idx / n, j = idx % n;
    W[(long)j * m + i] = A[(long)i * lda + j];
  }
  __syncthreads();
  // reflector of column j (rows j..m-1), formed by the wave that owns column j
  auto reflector = [&](int j) {
    double* v = W + (long)j * m;
    double loc = 0.0, xj = 0.0;
    for (int i = lane; i < m; i += 64) {
      if (i >= j) {
        const double x = v[i];
        loc += x * x;
        if (i == j) xj = x;
      }
    }
    const double s2 = wave_sum(loc);
    const double x0 = __shfl(xj, j % 64, 64);
    const double nrm = sqrt(s2);
    double tj = 0.0, alpha = 0.0, v0 = x0;
    if (nrm > 0.0) {
      alpha = x0 >= 0.0 ? -nrm : nrm;
      v0 = x0 - alpha;
      tj = 2.0 / (s2 - x0 * x0 + v0 * v0);
    }
    if (lane == j % 64) {
      v[j] = v0;
      tau[j] = tj;
      diag[j] = alpha;
    }
  };
  // w <- (I - tau v v^T) w over rows j..m-1
  auto apply = [&](const double* v, double tj, double* w, int j) {
    double part = 0.0;
    for (int i = lane; i < m; i += 64)
      if (i >= j) part += v[i] * w[i];
    const double f = tj * wave_sum(part);
    for (int i = lane; i < m; i += 64)
      if (i >= j) w[i] -= f * v[i];
  };
  if (c > 0 && wave == 0) reflector(0);
  __syncthreads();
  for (int j = 0; j < c; ++j) {
    const double tj = tau[j];
    const double* v = W + (long)j * m;
    const int nxt = j + 1;
    if (nxt < n && wave == nxt % NW) {
      if (tj != 0.0) apply(v, tj, W + (long)nxt * m, j);
      if (nxt < c) reflector(nxt);
    }
    if (tj != 0.0) {
      for (int col = nxt + 1; col < n; ++col)
        if (col % NW == wave) apply(v, tj, W + (long)col * m, j);
    }
    __syncthreads();
  }
  for (long idx = tid; idx < (long)c * n; idx += QR_NT) {
    const int i = idx / n, jj = idx % n;
    R[(long)i * ldr + jj] = jj < i ? 0.0 : (jj == i ? diag[i] : W[(long)jj * m + i]);
  }
  // Q = H_0 ... H_{c-1} E: column col of E is changed only by reflectors j <= col
  for (int col = wave; col < c; col += NW) {
    double* q = Qc + (long)col * m;
    for (int i = lane; i < m; i += 64) q[i] = (i == col) ? 1.0 : 0.0;
    for (int j = col; j >= 0; --j) {
      const double tj = tau[j];
      if (tj != 0.0) apply(W + (long)j * m, tj, q, j);
    }
  }
  __syncthreads();
  for (long idx = tid; idx < (long)m * c; idx += QR_NT) {
    const int i = idx / c, jj = idx % c;
    Q[(long)i * ldq + jj] = Qc[(long)jj * m + i];
  }
}

template <bool LDS>
__global__ __launch_bounds__(QR_NT) void qr_owner_kernel(int m, int n, const double* A, int lda, double* Q, int ldq,
                                                         double* R, int ldr, double* ws) {
  extern __shared__ double dyn[];
  qr_owner_body<LDS>(m, n, A, lda, Q, ldq, R, ldr, ws, dyn);
}

// One workgroup per job: the same QR as qr_owner_kernel for each job of the batch.
template <bool LDS>
__global__ __launch_bounds__(QR_NT) void qr_owner_batch_kernel(QrBatch b) {
  extern __shared__ double dyn[];
  const QrJob j = b.job[blockIdx.x];
  qr_owner_body<LDS>(j.m, j.n, j.A, j.lda, j.Q, j.ldq, j.R, j.ldr, j.ws, dyn);
}

// The same factorisation for matrices that do not fit in LDS (m <= 64 KR): W and the
// Q accumulation stay in global memory, with the same column ownership.  A column
// update loads the lane's KR rows of the column into registers at once (one memory
// latency per column rather than one per row block), takes the reflector from an LDS
// double buffer, and writes the column back once.  Column accesses are buffer
// loads / stores whose range is the column's m rows, so rows past m read as zero and
// are not written, with no branches (branches around each store make the compiler
// wait for every earlier store).  Reflector j is held in LDS with zeros outside rows
// j..m-1, so a column update needs no row masks: rows above j are left as they are.
// The owner of column j + 1 forms reflector j + 1 from its registers and publishes it
// in the other LDS buffer, so each column still costs one barrier.
// Q = H_0 ... H_{c-1} E is accumulated backwards: at step j every wave applies H_j to
// its columns col >= j (a column of E is untouched by the reflectors after it; rows
// above j are still zero), the reflector staged in LDS one step ahead by its owner.
typedef long long i64x1_t __attribute__((ext_vector_type(1)));

__device__ inline __amdgpu_buffer_rsrc_t column_rsrc(double* col, int m) {
  // raw buffer, 32-bit data format (the gfx9 descriptor word for untyped access)
  return __builtin_amdgcn_make_buffer_rsrc(col, (short)0, m * 8, 0x00020000);
}

// PAD = true: W and Q live in dynamic LDS (dyn) with the column stride padded to 64 KR
// rows of zeros, so column accesses are plain LDS reads and writes with no range
// checks; the padding rows stay zero (every reflector is zero there).
template <int KR, int NT, bool PAD>
__device__ __forceinline__ void qr_reg_body(int m, int n, const double* A, int lda, double* Q, int ldq, double* R,
                                            int ldr, double* ws, double* dyn) {
  constexpr int NW = NT / 64;
  __shared__ double sv[2][64 * KR];
  __shared__ double stau[2];
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int c = m < n ? m : n;
  const int ld = PAD ? 64 * KR : m;  // column stride of W and Q
  double* W = PAD ? dyn : ws;         // ld x n, column-major
  double* Qc = W + (long)ld * n;      // ld x c, column-major
  double* tau = Qc + (long)ld * c;    // c
  double* diag = tau + c;             // c
  if constexpr (PAD) {
    for (long idx = tid; idx < (long)ld * n; idx += NT) {
      const int i = idx % ld, j = idx / ld;
      W[(long)j * ld + i] = i < m ? A[(long)i * lda + j] : 0.0;
    }
  } else {
    for (long idx = tid; idx < (long)m * n; idx += NT) {
      const int i = idx / n, j = idx % n;
      W[(long)j * ld + i] = A[(long)i * lda + j];
    }
  }
  for (int i = tid; i < 2 * 64 * KR; i += NT) (&sv[0][0])[i] = 0.0;
  __syncthreads();
  double wr[KR];
  // all m rows of a column, rows below lo replaced by zero
  auto load_col = [&](double* w, int lo) {
    if constexpr (PAD) {
#pragma unroll
      for (int k = 0; k < KR; ++k) {
        const int i = lane + 64 * k;
        const double x = w[i];
        wr[k] = i >= lo ? x : 0.0;
      }
    } else {
      const __amdgpu_buffer_rsrc_t rs = column_rsrc(w, m);
#pragma unroll
      for (int k = 0; k < KR; ++k) {
        const int i = lane + 64 * k;
        const double x = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, lane * 8, 512 * k, 0));
        wr[k] = i >= lo ? x : 0.0;
      }
    }
  };
  auto store_col = [&](double* w) {
    if constexpr (PAD) {
#pragma unroll
      for (int k = 0; k < KR; ++k) w[lane + 64 * k] = wr[k];
    } else {
      const __amdgpu_buffer_rsrc_t rs = column_rsrc(w, m);
#pragma unroll
      for (int k = 0; k < KR; ++k)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(i64x1_t, wr[k]), rs, lane * 8, 512 * k, 0);
    }
  };
  // wr <- (I - tj v v^T) wr; v is zero outside the reflector's rows
  auto apply_reg = [&](const double* v, double tj) {
    double part = 0.0;
#pragma unroll
    for (int k = 0; k < KR; ++k) part += v[lane + 64 * k] * wr[k];
    const double f = tj * wave_sum(part);
    // read v again rather than holding it in KR more registers
    __asm__ volatile("" ::: "memory");
#pragma unroll
    for (int k = 0; k < KR; ++k) wr[k] -= f * v[lane + 64 * k];
  };
  // reflector of column j from wr (rows >= j, zero elsewhere): v to W column j and sv[buf]
  auto reflect = [&](int j, int buf) {
    double loc = 0.0, xj = 0.0;
#pragma unroll
    for (int k = 0; k < KR; ++k) {
      loc += wr[k] * wr[k];
      xj = lane + 64 * k == j ? wr[k] : xj;
    }
    const double s2 = wave_sum(loc);
    const double x0 = __shfl(xj, j % 64, 64);
    const double nrm = sqrt(s2);
    double tj = 0.0, alpha = 0.0, v0 = x0;
    if (nrm > 0.0) {
      alpha = x0 >= 0.0 ? -nrm : nrm;
      v0 = x0 - alpha;
      tj = 2.0 / (s2 - x0 * x0 + v0 * v0);
    }
#pragma unroll
    for (int k = 0; k < KR; ++k) sv[buf][lane + 64 * k] = lane + 64 * k == j ? v0 : wr[k];
    if (lane == j % 64) {
      W[(long)j * ld + j] = v0;
      tau[j] = tj;
      diag[j] = alpha;
      stau[buf] = tj;
    }
  };
  if (c > 0 && wave == 0) {
    load_col(W, 0);
    reflect(0, 0);
  }
  __syncthreads();
  for (int j = 0; j < c; ++j) {
    const double* v = sv[j & 1];
    const double tj = stau[j & 1];
    const int nxt = j + 1;
    if (nxt < n && wave == nxt % NW) {
      double* w = W + (long)nxt * ld;
      load_col(w, 0);
      if (tj != 0.0) apply_reg(v, tj);
      store_col(w);
      if (nxt < c) {
#pragma unroll
        for (int k = 0; k < KR; ++k) wr[k] = lane + 64 * k >= nxt ? wr[k] : 0.0;
        reflect(nxt, nxt & 1);
      }
    }
    if (tj != 0.0) {
      for (int col = nxt + 1; col < n; ++col) {
        if (col % NW != wave) continue;
        double* w = W + (long)col * ld;
        load_col(w, 0);
        apply_reg(v, tj);
        store_col(w);
      }
    }
    __syncthreads();
  }
  for (long idx = tid; idx < (long)c * n; idx += NT) {
    const int i = idx / n, jj = idx % n;
    R[(long)i * ldr + jj] = jj < i ? 0.0 : (jj == i ? diag[i] : W[(long)jj * ld + i]);
  }
  // Q, backwards over the reflectors; v_j staged into sv[j & 1] one step ahead
  auto stage = [&](int j) {
    load_col(W + (long)j * ld, j);
#pragma unroll
    for (int k = 0; k < KR; ++k) sv[j & 1][lane + 64 * k] = wr[k];
  };
  if (c > 0 && wave == (c - 1) % NW) stage(c - 1);
  __syncthreads();
  for (int j = c - 1; j >= 0; --j) {
    const double* v = sv[j & 1];
    const double tj = tau[j];
    for (int col = j; col < c; ++col) {
      if (col % NW != wave) continue;
      double* q = Qc + (long)col * ld;
      if (col == j) {
#pragma unroll
        for (int k = 0; k < KR; ++k) wr[k] = lane + 64 * k == j ? 1.0 : 0.0;
      } else {
        load_col(q, j + 1);  // rows up to j are still zero in this column
      }
      if (tj != 0.0) apply_reg(v, tj);
      store_col(q);
    }
    if (j > 0 && wave == (j - 1) % NW) stage(j - 1);
    __syncthreads();
  }
  for (long idx = tid; idx < (long)m * c; idx += NT) {
    const int i = idx / c, jj = idx % c;
    Q[(long)i * ldq + jj] = Qc[(long)jj * ld + i];
  }
}

// The same Householder QR with every column in registers for m <= 64 KR and
// n <= 16 CPW: column col is owned by wavefront col % 16 (slot col / 16), a lane holds
// rows lane, lane + 64, ... of each of its columns, so no column goes through memory
// while it is factored.  Step j: every wavefront applies reflector j (read from an LDS
// double buffer) to its columns right of j, the owner of column j + 1 first, which then
// forms reflector j + 1, publishes it in the other buffer and keeps it in place of its
// column below the diagonal (R above).  One barrier per column.  Reflectors also go to
// ws (column-major, stride m) for the accumulation of Q = H_0 ... H_{c-1} E, which runs
// backwards with the columns of Q in registers and each reflector staged into LDS two
// steps ahead (three buffers), so the L2 latency of the staging overlaps two steps.
// The arithmetic of a column does not depend on KR or CPW (padding rows are zero), so
// the batched launch, sized for its largest job, gives every job the results of its
// own launch.
constexpr int QRC_NT = 1024, QRC_NW = 16;

template <int KR, int CPW>
__device__ __forceinline__ void qr_cols_body(int m, int n, const double* A, int lda, double* Q, int ldq, double* R,
                                             int ldr, double* ws) {
  __shared__ double sv[3][64 * KR];
  __shared__ double stau[2];
  __shared__ double tau_s[QRC_NW * CPW], diag_s[QRC_NW * CPW];
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int c = m < n ? m : n;
  double w[CPW][KR];
#pragma unroll
  for (int s = 0; s < CPW; ++s) {
    const int col = wave + QRC_NW * s;
#pragma unroll
    for (int k = 0; k < KR; ++k) {
      const int i = lane + 64 * k;
      w[s][k] = (col < n && i < m) ? A[(long)i * lda + col] : 0.0;
    }
  }
  // w[s] <- (I - tj v v^T) w[s], v in LDS (zero outside the reflector's rows)
  auto apply = [&](int s, const double* v, double tj) {
    double part = 0.0;
#pragma unroll
    for (int k = 0; k < KR; ++k) part += v[lane + 64 * k] * w[s][k];
    const double f = tj * wave_sum(part);
#pragma unroll
    for (int k = 0; k < KR; ++k) w[s][k] -= f * v[lane + 64 * k];
  };
  // reflector of column j (slot s of this wavefront): rows >= j of w[s]
  auto reflect = [&](int j, int s, int buf) {
    double loc = 0.0, xj = 0.0;
#pragma unroll
    for (int k = 0; k < KR; ++k) {
      const int i = lane + 64 * k;
      const double x = i >= j ? w[s][k] : 0.0;
      loc += x * x;
      xj = i == j ? w[s][k] : xj;
    }
    const double s2 = wave_sum(loc);
    const double x0 = __shfl(xj, j % 64, 64);
    const double nrm = sqrt(s2);
    double tj = 0.0, alpha = 0.0, v0 = x0;
    if (nrm > 0.0) {
      alpha = x0 >= 0.0 ? -nrm : nrm;
      v0 = x0 - alpha;
      tj = 2.0 / (s2 - x0 * x0 + v0 * v0);
    }
    double* wsj = ws + (long)j * m;
#pragma unroll
    for (int k = 0; k < KR; ++k) {
      const int i = lane + 64 * k;
      const double v = i == j ? v0 : (i > j ? w[s][k] : 0.0);
      sv[buf][i] = v;
      if (i < m) wsj[i] = v;
      if (i == j) w[s][k] = v0;  // rows > j already hold v; rows < j keep R
    }
    if (lane == 0) {
      stau[buf] = tj;
      tau_s[j] = tj;
      diag_s[j] = alpha;
    }
  };
  if (c > 0 && wave == 0) reflect(0, 0, 0);
  __syncthreads();
  for (int j = 0; j < c; ++j) {
    const double* v = sv[j & 1];
    const double tj = stau[j & 1];
    const int nxt = j + 1;
    // the owner of column j + 1: that column first, then its reflector (slots are
    // compile-time indices, so the columns stay in registers)
#pragma unroll
    for (int s = 0; s < CPW; ++s) {
      if (nxt < n && wave + QRC_NW * s == nxt) {
        if (tj != 0.0) apply(s, v, tj);
        if (nxt < c) reflect(nxt, s, nxt & 1);
      }
    }
    if (tj != 0.0) {
#pragma unroll
      for (int s = 0; s < CPW; ++s) {
        const int col = wave + QRC_NW * s;
        if (col > nxt && col < n) apply(s, v, tj);
      }
    }
    __syncthreads();
  }
  // R: rows < col of a column are final, its diagonal is diag_s, zeros below
#pragma unroll
  for (int s = 0; s < CPW; ++s) {
    const int col = wave + QRC_NW * s;
    if (col >= n) continue;
#pragma unroll
    for (int k = 0; k < KR; ++k) {
      const int i = lane + 64 * k;
      if (i < c) R[(long)i * ldr + col] = i < col ? w[s][k] : (i == col ? diag_s[col] : 0.0);
    }
  }
  // Q = H_0 ... H_{c-1} E backwards; reflector j staged into sv[j % 3] two steps ahead
  auto stage = [&](int j) {
    const double* wsj = ws + (long)j * m;
#pragma unroll
    for (int k = 0; k < KR; ++k) {
      const int i = lane + 64 * k;
      sv[j % 3][i] = i < m ? wsj[i] : 0.0;
    }
  };
  __syncthreads();  // the reflectors in ws are complete (every wavefront wrote its own)
  if (wave == 0 && c >= 1) stage(c - 1);
  if (wave == 1 && c >= 2) stage(c - 2);
#pragma unroll
  for (int s = 0; s < CPW; ++s) {
    const int col = wave + QRC_NW * s;
#pragma unroll
    for (int k = 0; k < KR; ++k) w[s][k] = (lane + 64 * k == col) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int j = c - 1; j >= 0; --j) {
    if (j >= 2 && wave == j % QRC_NW) stage(j - 2);
    const double* v = sv[j % 3];
    const double tj = tau_s[j];
    if (tj != 0.0) {
#pragma unroll
      for (int s = 0; s < CPW; ++s) {
        const int col = wave + QRC_NW * s;
        if (col >= j && col < c) apply(s, v, tj);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int s = 0; s < CPW; ++s) {
    const int col = wave + QRC_NW * s;
    if (col >= c) continue;
#pragma unroll
    for (int k = 0; k < KR; ++k) {
      const int i = lane + 64 * k;
      if (i < m) Q[(long)i * ldq + col] = w[s][k];
    }
  }
}

template <int KR, int CPW>
__global__ __launch_bounds__(QRC_NT) void qr_cols_kernel(int m, int n, const double* A, int lda, double* Q, int ldq,
                                                         double* R, int ldr, double* ws) {
  qr_cols_body<KR, CPW>(m, n, A, lda, Q, ldq, R, ldr, ws);
}

template <int KR, int CPW>
__global__ __launch_bounds__(QRC_NT) void qr_cols_batch_kernel(QrBatch b) {
  const QrJob j = b.job[blockIdx.x];
  qr_cols_body<KR, CPW>(j.m, j.n, j.A, j.lda, j.Q, j.ldq, j.R, j.ldr, j.ws);
}

// rows per lane and columns per wavefront of the register-column QR (0: does not apply)
static int qrc_kr(int m) { return m <= 64 ? 1 : (m <= 128 ? 2 : (m <= 256 ? 4 : (m <= 512 ? 8 : 0))); }
static int qrc_cpw(int n) { return n <= 16 ? 1 : (n <= 32 ? 2 : (n <= 48 ? 3 : (n <= 80 ? 5 : 0))); }

template <int KR>
static void launch_qrc_kr(int cpw, const QrJob& j, const QrBatch* b, hipStream_t s) {
  if (b) {
    if (cpw == 1) hipLaunchKernelGGL((qr_cols_batch_kernel<KR, 1>), dim3(b->njob), dim3(QRC_NT), 0, s, *b);
    else if (cpw == 2) hipLaunchKernelGGL((qr_cols_batch_kernel<KR, 2>), dim3(b->njob), dim3(QRC_NT), 0, s, *b);
    else if (cpw == 3) hipLaunchKernelGGL((qr_cols_batch_kernel<KR, 3>), dim3(b->njob), dim3(QRC_NT), 0, s, *b);
    else hipLaunchKernelGGL((qr_cols_batch_kernel<KR, 5>), dim3(b->njob), dim3(QRC_NT), 0, s, *b);
  } else {
    if (cpw == 1)
      hipLaunchKernelGGL((qr_cols_kernel<KR, 1>), dim3(1), dim3(QRC_NT), 0, s, j.m, j.n, j.A, j.lda, j.Q, j.ldq, j.R,
                         j.ldr, j.ws);
    else if (cpw == 2)
      hipLaunchKernelGGL((qr_cols_kernel<KR, 2>), dim3(1), dim3(QRC_NT), 0, s, j.m, j.n, j.A, j.lda, j.Q, j.ldq, j.R,
                         j.ldr, j.ws);
    else if (cpw == 3)
      hipLaunchKernelGGL((qr_cols_kernel<KR, 3>), dim3(1), dim3(QRC_NT), 0, s, j.m, j.n, j.A, j.lda, j.Q, j.ldq, j.R,
                         j.ldr, j.ws);
    else
      hipLaunchKernelGGL((qr_cols_kernel<KR, 5>), dim3(1), dim3(QRC_NT), 0, s, j.m, j.n, j.A, j.lda, j.Q, j.ldq, j.R,
                         j.ldr, j.ws);
  }
}

// one QR (b == nullptr) or a batch sized for its largest job
static void launch_qrc(int kr, int cpw, const QrJob& j, const QrBatch* b, hipStream_t s) {
  if (kr == 1) launch_qrc_kr<1>(cpw, j, b, s);
  else if (kr == 2) launch_qrc_kr<2>(cpw, j, b, s);
  else if (kr == 4) launch_qrc_kr<4>(cpw, j, b, s);
  else launch_qrc_kr<8>(cpw, j, b, s);
}

// threads of the register variant: 32 rows per lane need the register file of 2 waves per SIMD
template <int KR>
constexpr int qr_reg_threads() { return KR >= 32 ? 512 : QR_NT; }

template <int KR, bool PAD>
__global__ __launch_bounds__(qr_reg_threads<KR>()) void qr_reg_kernel(int m, int n, const double* A, int lda,
                                                                     double* Q, int ldq, double* R, int ldr,
                                                                     double* ws) {
  extern __shared__ double dyn[];
  qr_reg_body<KR, qr_reg_threads<KR>(), PAD>(m, n, A, lda, Q, ldq, R, ldr, ws, dyn);
}

template <int KR, bool PAD>
__global__ __launch_bounds__(qr_reg_threads<KR>()) void qr_reg_batch_kernel(QrBatch b) {
  extern __shared__ double dyn[];
  const QrJob j = b.job[blockIdx.x];
  qr_reg_body<KR, qr_reg_threads<KR>(), PAD>(j.m, j.n, j.A, j.lda, j.Q, j.ldq, j.R, j.ldr, j.ws, dyn);
}

static void hip_check_attr(hipError_t e) {
  if (e != hipSuccess) throw Error(TNFEM_EDEVICE, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
}

// ----- blocked Householder QR for tall matrices (256 < m <= 2048, n >= 32) that do not fit in LDS
// Panels of nb columns: a panel is factored by one workgroup with the panel in LDS
// (wavefront w owns panel column w in registers, one barrier per column) and its
// compact-WY factor T (H_0 ... H_{nb-1} = I - V T V^T, T upper triangular from
// T_jj = tau_j, T[0:j, j] = -tau_j T[0:j, 0:j] V[:, 0:j]^T v_j) is formed; the trailing
// columns are then updated by many workgroups, A -= V T^T (V^T A), one wavefront per
// column with the panel's V staged in LDS.  Q = H_0 ... H_{c-1} E is accumulated
// backwards over the panels with Q -= V T (V^T Q) on columns j0.. of Q.  The storage
// follows the unblocked variants: W (m x n, column-major) holds R above the diagonal
// and the reflectors v (v_0 on the diagonal) below it; diag holds R's diagonal.
constexpr int QRB_NBMAX = 16;

__global__ void qr_to_colmajor_kernel(int m, int n, const double* A, int lda, double* W) {
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < (long)m * n; idx += (long)gridDim.x * blockDim.x) {
    const int i = idx / n, j = idx % n;
    W[(long)j * m + i] = A[(long)i * lda + j];
  }
}

__global__ void qr_identity_kernel(int m, int c, double* Qc) {
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < (long)m * c; idx += (long)gridDim.x * blockDim.x)
    Qc[idx] = (idx % m == idx / m) ? 1.0 : 0.0;
}

__global__ void qr_outputs_kernel(int m, int n, const double* W, const double* Qc, const double* diag, double* Q, int ldq,
                                  double* R, int ldr) {
  const int c = m < n ? m : n;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < (long)c * n; idx += (long)gridDim.x * blockDim.x) {
    const int i = idx / n, jj = idx % n;
    R[(long)i * ldr + jj] = jj < i ? 0.0 : (jj == i ? diag[i] : W[(long)jj * m + i]);
  }
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < (long)m * c; idx += (long)gridDim.x * blockDim.x) {
    const int i = idx / c, jj = idx % c;
    Q[(long)i * ldq + jj] = Qc[(long)jj * m + i];
  }
}

// Panel columns j0 .. j0 + nbk - 1 (nbk <= 16), rows j0 .. m - 1 (at most 64 KR).
template <int KR>
__global__ __launch_bounds__(1024) void qr_panel_kernel(int m, int j0, int nbk, double* W, double* tau, double* diag,
                                                       double* Tk) {
  constexpr int LDV = 64 * KR;
  extern __shared__ double sh[];
  double* Vp = sh;                         // nbk x LDV: reflector a in Vp[a * LDV + (i - j0)]
  __shared__ double G[QRB_NBMAX][QRB_NBMAX];
  __shared__ double stau[QRB_NBMAX];
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int mr = m - j0;
  double wr[KR];
  double* col = W + (long)(j0 + wave) * m + j0;  // rows j0.. of the wave's panel column
  if (wave < nbk) {
    const __amdgpu_buffer_rsrc_t rs = column_rsrc(col, mr);
#pragma unroll
    for (int k = 0; k < KR; ++k)
      wr[k] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, lane * 8, 512 * k, 0));
  }
  for (int j = 0; j < nbk; ++j) {
    if (wave == j) {
      // reflector of local column j from rows j.. (rows above are R entries, kept in wr)
      double loc = 0.0, xj = 0.0;
#pragma unroll
      for (int k = 0; k < KR; ++k) {
        const int i = lane + 64 * k;
        const double x = i >= j ? wr[k] : 0.0;
        loc += x * x;
        xj = i == j ? wr[k] : xj;
      }
      const double s2 = wave_sum(loc);
      const double x0 = __shfl(xj, j % 64, 64);
      const double nrm = sqrt(s2);
      double tj = 0.0, alpha = 0.0, v0 = x0;
      if (nrm > 0.0) {
        alpha = x0 >= 0.0 ? -nrm : nrm;
        v0 = x0 - alpha;
        tj = 2.0 / (s2 - x0 * x0 + v0 * v0);
      }
#pragma unroll
      for (int k = 0; k < KR; ++k) {
        const int i = lane + 64 * k;
        wr[k] = i == j ? v0 : wr[k];
        Vp[j * LDV + i] = i >= j ? wr[k] : 0.0;  // rows >= mr read as zero from the load
      }
      const __amdgpu_buffer_rsrc_t rs = column_rsrc(col, mr);
#pragma unroll
      for (int k = 0; k < KR; ++k)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(i64x1_t, wr[k]), rs, lane * 8, 512 * k, 0);
      if (lane == 0) {
        tau[j0 + j] = tj;
        diag[j0 + j] = alpha;
        stau[j] = tj;
      }
    }
    __syncthreads();
    if (wave > j && wave < nbk && stau[j] != 0.0) {
      const double* v = Vp + j * LDV;
      double part = 0.0;
#pragma unroll
      for (int k = 0; k < KR; ++k) part += v[lane + 64 * k] * wr[k];
      const double f = stau[j] * wave_sum(part);
      __asm__ volatile("" ::: "memory");
#pragma unroll
      for (int k = 0; k < KR; ++k) wr[k] -= f * v[lane + 64 * k];
    }
  }
  // G = V^T V (row a by wavefront a), then T by rows: lane r of wavefront 0 holds row r
  if (wave < nbk) {
    for (int b = 0; b < nbk; ++b) {
      double part = 0.0;
#pragma unroll
      for (int k = 0; k < KR; ++k) part += Vp[wave * LDV + lane + 64 * k] * Vp[b * LDV + lane + 64 * k];
      const double g = wave_sum(part);
      if (lane == 0) G[wave][b] = g;
    }
  }
  __syncthreads();
  if (wave == 0) {
    const int r = lane;
    double trow[QRB_NBMAX];
#pragma unroll
    for (int s = 0; s < QRB_NBMAX; ++s) trow[s] = 0.0;
#pragma unroll
    for (int j = 0; j < QRB_NBMAX; ++j) {
      if (j < nbk) {
        double acc = 0.0;
#pragma unroll
        for (int s = 0; s < QRB_NBMAX; ++s)
          if (s >= r && s < j) acc += trow[s] * G[s][j];
        trow[j] = r < j ? -stau[j] * acc : (r == j ? stau[j] : 0.0);
      }
    }
    if (r < nbk)
      for (int s = 0; s < nbk; ++s) Tk[r * QRB_NBMAX + s] = trow[s];
  }
}

// A[j0.., cols] -= V M (V^T A[j0.., cols]) with M = T^T (trans = 1) or T (trans = 0);
// A column-major with column stride m; columns col0 .. col0 + ncols - 1; one wavefront
// per column, four per workgroup; V (rows j0.., nbk columns) staged in LDS from W.
template <int KR>
__global__ __launch_bounds__(256) void qr_wy_update_kernel(int m, int j0, int nbk, const double* W, double* A, int col0,
                                                          int ncols, const double* Tk, int trans) {
  constexpr int LDV = 64 * KR;
  extern __shared__ double sh[];
  double* Vp = sh;
  __shared__ double T[QRB_NBMAX][QRB_NBMAX];
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int mr = m - j0;
  for (int idx = tid; idx < nbk * LDV; idx += 256) {
    const int a = idx / LDV, i = idx % LDV;
    // reflector a: zero above its diagonal row a, v_0 on it, v below; zero past the matrix
    Vp[idx] = (i >= a && i < mr) ? W[(long)(j0 + a) * m + j0 + i] : 0.0;
  }
  for (int idx = tid; idx < QRB_NBMAX * QRB_NBMAX; idx += 256) {
    const int r = idx / QRB_NBMAX, s2 = idx % QRB_NBMAX;
    T[r][s2] = (r < nbk && s2 < nbk) ? Tk[r * QRB_NBMAX + s2] : 0.0;
  }
  __syncthreads();
  const int cl = blockIdx.x * 4 + wave;
  if (cl >= ncols) return;
  double* a = A + (long)(col0 + cl) * m + j0;
  const __amdgpu_buffer_rsrc_t rs = column_rsrc(a, mr);
  double ar[KR];
#pragma unroll
  for (int k = 0; k < KR; ++k)
    ar[k] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, lane * 8, 512 * k, 0));
  double y[QRB_NBMAX];
#pragma unroll
  for (int b = 0; b < QRB_NBMAX; ++b) {
    double part = 0.0;
    if (b < nbk) {
#pragma unroll
      for (int k = 0; k < KR; ++k) part += Vp[b * LDV + lane + 64 * k] * ar[k];
    }
    y[b] = wave_sum(part);
  }
  double z[QRB_NBMAX];
#pragma unroll
  for (int r = 0; r < QRB_NBMAX; ++r) {
    double acc = 0.0;
#pragma unroll
    for (int b = 0; b < QRB_NBMAX; ++b) acc += (trans ? T[b][r] : T[r][b]) * y[b];
    z[r] = acc;
  }
#pragma unroll
  for (int k = 0; k < KR; ++k) {
    double acc = 0.0;
#pragma unroll
    for (int b = 0; b < QRB_NBMAX; ++b) acc += Vp[b * LDV + lane + 64 * k] * z[b];
    ar[k] -= acc;
  }
#pragma unroll
  for (int k = 0; k < KR; ++k)
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(i64x1_t, ar[k]), rs, lane * 8, 512 * k, 0);
}

static int qrb_blocks(long n) { return (int)std::min<long>(std::max<long>((n + 255) / 256, 1), 2048); }

template <int KR>
static void qr_blocked_kr(int m, int n, const double* A, int lda, double* Q, int ldq, double* R, int ldr, double* ws,
                          hipStream_t s) {
  constexpr int LDV = 64 * KR;
  const int nb = KR >= 32 ? 8 : QRB_NBMAX;  // panel in LDS: nb x 64 KR doubles <= 128 KB
  const int c = m < n ? m : n;
  double* W = ws;
  double* Qc = W + (long)m * n;
  double* tau = Qc + (long)m * c;
  double* diag = tau + c;
  double* T = diag + c;  // one QRB_NBMAX x QRB_NBMAX block per panel
  const size_t panel_lds = (size_t)nb * LDV * sizeof(double);
  static std::once_flag once;
  std::call_once(once, [] {
    hip_check_attr(hipFuncSetAttribute(reinterpret_cast<const void*>(&qr_panel_kernel<KR>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 1024));
    hip_check_attr(hipFuncSetAttribute(reinterpret_cast<const void*>(&qr_wy_update_kernel<KR>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 1024));
  });
  hipLaunchKernelGGL(qr_to_colmajor_kernel, dim3(qrb_blocks((long)m * n)), dim3(256), 0, s, m, n, A, lda, W);
  const int npanel = (c + nb - 1) / nb;
  for (int k = 0; k < npanel; ++k) {
    const int j0 = k * nb, nbk = std::min(nb, c - j0);
    hipLaunchKernelGGL(qr_panel_kernel<KR>, dim3(1), dim3(1024), panel_lds, s, m, j0, nbk, W, tau, diag,
                       T + (long)k * QRB_NBMAX * QRB_NBMAX);
    const int rest = n - (j0 + nbk);
    if (rest > 0)
      hipLaunchKernelGGL(qr_wy_update_kernel<KR>, dim3((rest + 3) / 4), dim3(256), panel_lds, s, m, j0, nbk, W, W,
                         j0 + nbk, rest, T + (long)k * QRB_NBMAX * QRB_NBMAX, 1);
  }
  hipLaunchKernelGGL(qr_identity_kernel, dim3(qrb_blocks((long)m * c)), dim3(256), 0, s, m, c, Qc);
  for (int k = npanel - 1; k >= 0; --k) {
    const int j0 = k * nb, nbk = std::min(nb, c - j0);
    const int cols = c - j0;
    hipLaunchKernelGGL(qr_wy_update_kernel<KR>, dim3((cols + 3) / 4), dim3(256), panel_lds, s, m, j0, nbk, W, Qc, j0,
                       cols, T + (long)k * QRB_NBMAX * QRB_NBMAX, 0);
  }
  hipLaunchKernelGGL(qr_outputs_kernel, dim3(qrb_blocks((long)m * std::max(n, c))), dim3(256), 0, s, m, n, W, Qc,
                     diag, Q, ldq, R, ldr);
}

// whether the blocked QR takes this shape (when it does not fit in LDS)
static bool qr_blocked_ok(int m, int n) { return m > 256 && m <= 2048 && std::min(m, n) >= 32; }

size_t qr_ws_doubles(int m, int n) {
  const size_t c = (size_t)std::min(m, n);
  return (size_t)m * n + (size_t)m * c + 2 * c + (c / 8 + 1) * QRB_NBMAX * QRB_NBMAX;
}

static void launch_qr_blocked(int m, int n, const double* A, int lda, double* Q, int ldq, double* R, int ldr,
                              double* ws, hipStream_t s) {
  if (m <= 512) qr_blocked_kr<8>(m, n, A, lda, Q, ldq, R, ldr, ws, s);
  else if (m <= 1024) qr_blocked_kr<16>(m, n, A, lda, Q, ldq, R, ldr, ws, s);
  else qr_blocked_kr<32>(m, n, A, lda, Q, ldq, R, ldr, ws, s);
}

// rows per lane of the register variant for m rows (0: too tall, use the plain global variant)
static int qr_reg_rows(int m) { return m <= 512 ? 8 : (m <= 1024 ? 16 : (m <= 2048 ? 32 : 0)); }
// rows per lane of the padded LDS variant (0: not offered for this height)
static int qr_pad_rows(int m) { return m <= 64 ? 1 : (m <= 128 ? 2 : (m <= 256 ? 4 : (m <= 512 ? 8 : 0))); }

static size_t qr_lds_bytes(int m, int n) {
  const int c = m < n ? m : n;
  return ((size_t)m * n + (size_t)m * c + 2 * (size_t)c) * sizeof(double);
}
// dynamic LDS of the padded variant with kr rows per lane (its reflector buffers are static)
static size_t qr_pad_bytes(int m, int n, int kr) {
  const int c = m < n ? m : n;
  const size_t ld = 64 * (size_t)kr;
  return (ld * n + ld * c + 2 * (size_t)c) * sizeof(double);
}
static bool qr_pad_fits(int m, int n, int kr) {
  return kr > 0 && qr_pad_bytes(m, n, kr) + 2 * 64 * (size_t)kr * sizeof(double) + 64 <= QR_LDS_BYTES;
}

// the kernels' static LDS (reflector buffers) counts against the same 160 KB, so the
// dynamic limit is what qr_pad_fits allows
template <int KR, bool PAD>
static void qr_reg_attr() {
  static std::once_flag once;
  std::call_once(once, [] {
    const int dyn = (int)(QR_LDS_BYTES - 2 * 64 * (size_t)KR * sizeof(double) - 64);
    hip_check_attr(hipFuncSetAttribute(reinterpret_cast<const void*>(&qr_reg_kernel<KR, PAD>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, dyn));
    hip_check_attr(hipFuncSetAttribute(reinterpret_cast<const void*>(&qr_reg_batch_kernel<KR, PAD>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, dyn));
  });
}

template <int KR, bool PAD>
static void launch_qr_reg_batch(const QrBatch& b, size_t lds, hipStream_t s) {
  if (PAD) qr_reg_attr<KR, PAD>();
  hipLaunchKernelGGL((qr_reg_batch_kernel<KR, PAD>), dim3(b.njob), dim3(qr_reg_threads<KR>()), lds, s, b);
}

void launch_qr_batch(const std::vector<QrJob>& jobs, hipStream_t s) {
  if (jobs.size() > (size_t)QR_BATCH_MAX) throw Error(TNFEM_EINVAL, "QR batch: too many jobs");
  for (const QrJob& j : jobs)
    if (j.ws_cap < qr_ws_doubles(j.m, j.n))
      throw Error(TNFEM_EINVAL, "QR batch: workspace of " + std::to_string(j.ws_cap) + " doubles below the " +
                                    std::to_string(qr_ws_doubles(j.m, j.n)) + " a " + std::to_string(j.m) + " x " +
                                    std::to_string(j.n) + " QR may use");
  static std::once_flag attr_once;
  std::call_once(attr_once, [] {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&qr_owner_batch_kernel<true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)QR_LDS_BYTES);
  });
  // the register-column kernel for the jobs it takes (one launch sized for the largest),
  // then the padded LDS variant for the jobs that fit with the batch's common row count
  // per lane, then the unpadded LDS kernel, then the global-memory variants
  QrBatch in_cols;
  int ckr = 0, ccpw = 0;
  std::vector<QrJob> rest_jobs;
  for (const QrJob& j : jobs) {
    if (qrc_kr(j.m) > 0 && qrc_cpw(j.n) > 0) {
      in_cols.job[in_cols.njob++] = j;
      ckr = std::max(ckr, qrc_kr(j.m));
      ccpw = std::max(ccpw, qrc_cpw(j.n));
    } else {
      rest_jobs.push_back(j);
    }
  }
  if (in_cols.njob) {
    launch_qrc(ckr, ccpw, in_cols.job[0], &in_cols, s);
    TN_CHECK_LAUNCH();
  }
  int kp = 0;
  for (const QrJob& j : rest_jobs) kp = std::max(kp, qr_pad_rows(j.m) == 0 ? 1 << 20 : qr_pad_rows(j.m));
  QrBatch in_pad, in_lds, in_ws;
  size_t pad_max = 0, lds_max = 0;
  for (const QrJob& j : rest_jobs) {
    if (kp <= 8 && qr_pad_fits(j.m, j.n, kp)) {
      in_pad.job[in_pad.njob++] = j;
      pad_max = std::max(pad_max, qr_pad_bytes(j.m, j.n, kp));
    } else if (qr_lds_bytes(j.m, j.n) <= QR_LDS_BYTES) {
      in_lds.job[in_lds.njob++] = j;
      lds_max = std::max(lds_max, qr_lds_bytes(j.m, j.n));
    } else {
      in_ws.job[in_ws.njob++] = j;
    }
  }
  if (in_pad.njob) {
    if (kp == 1) launch_qr_reg_batch<1, true>(in_pad, pad_max, s);
    else if (kp == 2) launch_qr_reg_batch<2, true>(in_pad, pad_max, s);
    else if (kp == 4) launch_qr_reg_batch<4, true>(in_pad, pad_max, s);
    else launch_qr_reg_batch<8, true>(in_pad, pad_max, s);
    TN_CHECK_LAUNCH();
  }
  if (in_lds.njob) {
    hipLaunchKernelGGL(qr_owner_batch_kernel<true>, dim3(in_lds.njob), dim3(QR_NT), lds_max, s, in_lds);
    TN_CHECK_LAUNCH();
  }
  if (in_ws.njob) {
    // tall jobs take the blocked QR one after another; the rest share one launch
    QrBatch rest;
    for (int i = 0; i < in_ws.njob; ++i) {
      const QrJob& j = in_ws.job[i];
      if (qr_blocked_ok(j.m, j.n)) launch_qr_blocked(j.m, j.n, j.A, j.lda, j.Q, j.ldq, j.R, j.ldr, j.ws, s);
      else rest.job[rest.njob++] = j;
    }
    in_ws = rest;
  }
  if (in_ws.njob) {
    int kr = 8;
    for (int i = 0; i < in_ws.njob; ++i) {
      const int r = qr_reg_rows(in_ws.job[i].m);
      kr = r == 0 ? 0 : (kr == 0 ? 0 : std::max(kr, r));
    }
    if (kr == 8) launch_qr_reg_batch<8, false>(in_ws, 0, s);
    else if (kr == 16) launch_qr_reg_batch<16, false>(in_ws, 0, s);
    else if (kr == 32) launch_qr_reg_batch<32, false>(in_ws, 0, s);
    else hipLaunchKernelGGL(qr_owner_batch_kernel<false>, dim3(in_ws.njob), dim3(QR_NT), 0, s, in_ws);
    TN_CHECK_LAUNCH();
  }
}

template <int KR, bool PAD>
static void launch_qr_reg(int m, int n, const double* A, int lda, double* Q, int ldq, double* R, int ldr,
                          double* ws, size_t lds, hipStream_t s) {
  if (PAD) qr_reg_attr<KR, PAD>();
  hipLaunchKernelGGL((qr_reg_kernel<KR, PAD>), dim3(1), dim3(qr_reg_threads<KR>()), lds, s, m, n, A, lda, Q, ldq,
                     R, ldr, ws);
}

void launch_qr(int m, int n, const double* A, int lda, double* Q, int ldq, double* R, int ldr, double* ws,
               size_t ws_cap, hipStream_t s) {
  if (ws_cap < qr_ws_doubles(m, n))
    throw Error(TNFEM_EINVAL, "QR: workspace of " + std::to_string(ws_cap) + " doubles below the " +
                                  std::to_string(qr_ws_doubles(m, n)) + " a " + std::to_string(m) + " x " +
                                  std::to_string(n) + " QR may use");
  const size_t bytes = qr_lds_bytes(m, n);
  const int kp = qr_pad_rows(m);
  if (qrc_kr(m) > 0 && qrc_cpw(n) > 0) {
    QrJob j{m, n, lda, ldq, ldr, A, Q, R, ws, ws_cap};
    launch_qrc(qrc_kr(m), qrc_cpw(n), j, nullptr, s);
  } else if (qr_pad_fits(m, n, kp)) {
    const size_t pb = qr_pad_bytes(m, n, kp);
    if (kp == 1) launch_qr_reg<1, true>(m, n, A, lda, Q, ldq, R, ldr, ws, pb, s);
    else if (kp == 2) launch_qr_reg<2, true>(m, n, A, lda, Q, ldq, R, ldr, ws, pb, s);
    else if (kp == 4) launch_qr_reg<4, true>(m, n, A, lda, Q, ldq, R, ldr, ws, pb, s);
    else launch_qr_reg<8, true>(m, n, A, lda, Q, ldq, R, ldr, ws, pb, s);
  } else if (bytes <= QR_LDS_BYTES) {
    static std::once_flag attr_once;
    std::call_once(attr_once, [] {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&qr_owner_kernel<true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)QR_LDS_BYTES);
    });
    hipLaunchKernelGGL(qr_owner_kernel<true>, dim3(1), dim3(QR_NT), bytes, s, m, n, A, lda, Q, ldq, R, ldr, ws);
  } else if (qr_blocked_ok(m, n)) {
    launch_qr_blocked(m, n, A, lda, Q, ldq, R, ldr, ws, s);
  } else {
    const int kr = qr_reg_rows(m);
    if (kr == 8) launch_qr_reg<8, false>(m, n, A, lda, Q, ldq, R, ldr, ws, 0, s);
    else if (kr == 16) launch_qr_reg<16, false>(m, n, A, lda, Q, ldq, R, ldr, ws, 0, s);
    else if (kr == 32) launch_qr_reg<32, false>(m, n, A, lda, Q, ldq, R, ldr, ws, 0, s);
    else hipLaunchKernelGGL(qr_owner_kernel<false>, dim3(1), dim3(QR_NT), 0, s, m, n, A, lda, Q, ldq, R, ldr, ws);
  }
  TN_CHECK_LAUNCH();
}

// ----------------------------------------------------------------------------- Jacobi SVD

// Jacobi rotation of a column pair with squared norms a, b and inner product c:
// tan(theta) = t, the root of smaller magnitude of t^2 + 2 zeta t - 1 = 0 with
// zeta = (b - a) / (2c), cs = 1 / sqrt(1 + t^2), sn = cs t.  The reciprocals and
// square roots are the hardware approximations refined by two Newton steps each
// (quadratic convergence from their ~26 correct bits), a shorter dependency chain
// than IEEE division and square root; the rotation only needs a few ulps.
__device__ inline double rcp_refined(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = fma(y, fma(-x, y, 1.0), y);
  return fma(y, fma(-x, y, 1.0), y);
}
__device__ inline double rsq_refined(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  return fma(0.5 * y, fma(-x * y, y, 1.0), y);
}
// c != 0 and a, b >= 0
__device__ inline void jacobi_rotation(double a, double b, double c, double& cs, double& sn) {
  const double zeta = (b - a) * rcp_refined(2.0 * c);
  const double az = fabs(zeta);
  double t;
  if (az < 1e150) {
    const double x = fma(zeta, zeta, 1.0);
    t = rcp_refined(az + x * rsq_refined(x));
  } else {
    t = 0.5 / az;
  }
  t = zeta >= 0.0 ? t : -t;
  cs = rsq_refined(fma(t, t, 1.0));
  sn = cs * t;
}
// whether the pair is off the rounding level: |c| > eps sqrt(a b)
__device__ inline bool jacobi_rotate(double a, double b, double c, double eps) {
  return c != 0.0 && c * c > eps * eps * (a * b);
}

constexpr int SV_NT = 256;
constexpr int SV_LDS_MAXN = 64;
constexpr int SV_MAXN = 256;

__global__ __launch_bounds__(SV_NT) void jacobi_svd_kernel(int n, const double* G, int ldg, int trans, double* U, double* S,
                                                           double* V, double* ws) {
  __shared__ double lds[2 * SV_LDS_MAXN * SV_LDS_MAXN];
  __shared__ double sv[SV_MAXN];
  __shared__ int pos[SV_MAXN];
  __shared__ int rotated;
  const int tid = threadIdx.x;
  const bool use_lds = n <= SV_LDS_MAXN;
  double* Gc = use_lds ? lds : ws;                      // column-major n x n
  double* Vc = use_lds ? lds + n * n : ws + (long)n * n;
  for (int idx = tid; idx < n * n; idx += SV_NT) {
    const int i = idx % n, j = idx / n;
    Gc[idx] = trans ? G[(long)j * ldg + i] : G[(long)i * ldg + j];
    Vc[idx] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int npad = n + (n & 1);
  const int npairs = npad / 2;
  int tpp = SV_NT / (npairs > 0 ? npairs : 1);
  if (tpp > 64) tpp = 64;
  int pw = 1;
  while (pw * 2 <= tpp) pw *= 2;
  tpp = pw;
  const int pair = tid / tpp, sub = tid % tpp;
  // rotation threshold at the rounding level of an n-term dot product: smaller
  // off-diagonal values are rounding noise, and rotating them never terminates
  const double eps = (n > 4 ? n : 4) * 2.220446049250313e-16;
  for (int sweep = 0; sweep < 40 && n > 1; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int step = 0; step < npad - 1; ++step) {
      if (pair < npairs) {
        // circle method: position 0 fixed, others rotate
        const int ia = pair, ib = npad - 1 - pair;
        const int pa = ia == 0 ? 0 : 1 + (ia - 1 + step) % (npad - 1);
        const int pb = ib == 0 ? 0 : 1 + (ib - 1 + step) % (npad - 1);
        const int p = pa < pb ? pa : pb, q = pa < pb ? pb : pa;
        double a = 0.0, b = 0.0, cc = 0.0;
        if (q < n) {
          for (int i = sub; i < n; i += tpp) {
            const double gp = Gc[p * n + i], gq = Gc[q * n + i];
            a += gp * gp;
            b += gq * gq;
            cc += gp * gq;
          }
        }
        a = group_sum(a, tpp);
        b = group_sum(b, tpp);
        cc = group_sum(cc, tpp);
        if (q < n && jacobi_rotate(a, b, cc, eps)) {
          double cs, sn;
          jacobi_rotation(a, b, cc, cs, sn);
          for (int i = sub; i < n; i += tpp) {
            const double gp = Gc[p * n + i], gq = Gc[q * n + i];
            Gc[p * n + i] = cs * gp - sn * gq;
            Gc[q * n + i] = sn * gp + cs * gq;
            const double vp = Vc[p * n + i], vq = Vc[q * n + i];
            Vc[p * n + i] = cs * vp - sn * vq;
            Vc[q * n + i] = sn * vp + cs * vq;
          }
          if (sub == 0) rotated = 1;
        }
      }
      __syncthreads();
    }
    const int any = rotated;
    __syncthreads();
    if (!any) break;
  }
  for (int j = tid; j < n; j += SV_NT) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += Gc[j * n + i] * Gc[j * n + i];
    sv[j] = sqrt(s);
  }
  __syncthreads();
  for (int j = tid; j < n; j += SV_NT) {
    int r = 0;
    for (int i = 0; i < n; ++i) r += (sv[i] > sv[j]) || (sv[i] == sv[j] && i < j);
    pos[j] = r;
  }
  __syncthreads();
  for (long idx = tid; idx < (long)n * n; idx += SV_NT) {
    const int j = idx / n, i = idx % n;  // column j of the unsorted factors, row i
    const int pj = pos[j];
    const double s = sv[j];
    U[(long)i * n + pj] = s > 0.0 ? Gc[j * n + i] / s : (i == pj ? 1.0 : 0.0);
    V[(long)i * n + pj] = Vc[j * n + i];
  }
  for (int j = tid; j < n; j += SV_NT) S[pos[j]] = sv[j];
}

// The same one-sided Jacobi iteration for n <= 64 (n <= 128 without V).  Each
// column pair of a step is owned by an aligned group of SVW_TPP lanes of one
// wavefront; lane `sub` of a group holds rows sub, sub + SVW_TPP, ... of both
// columns in registers from the dot products to the rotation, and the group
// reduces with DPP sums.  Rows are
// zero-padded to NR = SVW_TPP * RPL (no bounds tests in the step loop; zero rows
// and the zero padding column of an odd n never rotate).  The column stride LD is
// congruent to SVW_TPP mod 32 doubles: the groups of a half-wave read consecutive
// columns of the round-robin schedule and so hit disjoint LDS banks.
// WITH_V: a second set of wavefronts applies each step's rotations to V one step
// behind the G wavefronts (rotation parameters through LDS), off the critical path
// of the next step's dot products.  Without V the kernel returns the normalised
// columns of G (its left singular vectors) and S only.
// Dynamic LDS: svw_lds_bytes(n, RPL, WITH_V).
constexpr int SVW_MAXN = 64;        // with V (G and V in LDS)
constexpr int SVW_MAXN_LEFT = 128;  // without V (G alone in LDS)
constexpr int SVW_TPP = 8;
constexpr int SVW_MAX_THREADS = 512;

__host__ __device__ constexpr int svw_ld(int rpl) {
  return SVW_TPP * rpl + ((SVW_TPP - SVW_TPP * rpl) % 32 + 32) % 32;
}
__host__ __device__ inline int svw_npairs(int n) {
  const int npad = n + (n & 1);
  return npad / 2 > 0 ? npad / 2 : 1;
}
// G wavefronts: whole waves covering npairs groups of SVW_TPP lanes
__host__ __device__ inline int svw_gthreads(int n) { return (svw_npairs(n) * SVW_TPP + 63) / 64 * 64; }
static int svw_rpl(int n) {
  return n <= SVW_TPP ? 1 : n <= 2 * SVW_TPP ? 2 : n <= 4 * SVW_TPP ? 4 : n <= 8 * SVW_TPP ? 8 : 16;
}
static size_t svw_lds_bytes(int n, int rpl, bool with_v) {
  const size_t npad = n + (n & 1);
  const size_t cols = (with_v ? 2 : 1) * npad * svw_ld(rpl);
  return (cols + (with_v ? 4 * svw_npairs(n) : 0) + npad) * sizeof(double) + npad * sizeof(int);
}
static int svw_threads(int n, bool with_v) { return (with_v ? 2 : 1) * svw_gthreads(n); }

template <int RPL, bool WITH_V>
__device__ __forceinline__ void jacobi_svd_wave_body(int n, const double* G, int ldg, int trans, double* U, double* S,
                                                     double* V, double* dyn) {
  constexpr int TPP = SVW_TPP, NR = TPP * RPL, LD = svw_ld(RPL);
  const int npad = n + (n & 1);
  const int npairs = svw_npairs(n);
  const int ngt = svw_gthreads(n);
  double* Gc = dyn;                                    // npad columns of stride LD
  double* Vc = Gc + (long)npad * LD;                   // WITH_V
  double* rotb = Vc + (WITH_V ? (long)npad * LD : 0);  // WITH_V: (cs, sn) per pair, two steps
  double* sv = rotb + (WITH_V ? 4 * npairs : 0);
  int* pos = reinterpret_cast<int*>(sv + npad);
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int idx = tid; idx < npad * NR; idx += nt) {
    const int i = idx % NR, j = idx / NR;
    Gc[j * LD + i] = (i < n && j < n) ? (trans ? G[(long)j * ldg + i] : G[(long)i * ldg + j]) : 0.0;
    if (WITH_V) Vc[j * LD + i] = (i == j && j < n) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int m1 = npad - 1;
  // rotation threshold at the rounding level of an n-term dot product: smaller
  // off-diagonal values are rounding noise, and rotating them never terminates
  const double eps = (n > 4 ? n : 4) * 2.220446049250313e-16;
  const bool isg = !WITH_V || tid < ngt;
  const int gt = isg ? tid : tid - ngt;
  const int pair = gt / TPP, sub = gt % TPP;
  const bool live = pair < npairs;
  const int ia = pair, ib = npad - 1 - pair;
  int buf = 0;
  int vpa = -1, vpb = -1;  // V wavefronts: the columns of the step still to apply
  for (int sweep = 0; sweep < 40 && n > 1; ++sweep) {
    int rot = 0;
    int pa = ia, pb = ib;  // round-robin positions; pair 0 keeps column 0
    for (int step = 0; step < m1; ++step) {
      if (isg) {
        if (live) {
          double gp[RPL], gq[RPL];
#pragma unroll
          for (int r = 0; r < RPL; ++r) {
            gp[r] = Gc[pa * LD + sub + r * TPP];
            gq[r] = Gc[pb * LD + sub + r * TPP];
          }
          double a = 0.0, b = 0.0, c = 0.0;
#pragma unroll
          for (int r = 0; r < RPL; ++r) {
            a = fma(gp[r], gp[r], a);
            b = fma(gq[r], gq[r], b);
            c = fma(gp[r], gq[r], c);
          }
          a += dpp_get<DPP_XOR1>(a);
          b += dpp_get<DPP_XOR1>(b);
          c += dpp_get<DPP_XOR1>(c);
          a += dpp_get<DPP_XOR2>(a);
          b += dpp_get<DPP_XOR2>(b);
          c += dpp_get<DPP_XOR2>(c);
          a += dpp_get<DPP_HALF_MIRROR>(a);
          b += dpp_get<DPP_HALF_MIRROR>(b);
          c += dpp_get<DPP_HALF_MIRROR>(c);
          double cs = 1.0, sn = 0.0;
          if (jacobi_rotate(a, b, c, eps)) {
            jacobi_rotation(a, b, c, cs, sn);
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
              Gc[pa * LD + sub + r * TPP] = cs * gp[r] - sn * gq[r];
              Gc[pb * LD + sub + r * TPP] = sn * gp[r] + cs * gq[r];
            }
            rot = 1;
          }
          if (WITH_V && sub == 0) {
            rotb[2 * (buf * npairs + pair)] = cs;
            rotb[2 * (buf * npairs + pair) + 1] = sn;
          }
        }
      } else if (live && vpa >= 0) {
        const double cs = rotb[2 * ((buf ^ 1) * npairs + pair)];
        const double sn = rotb[2 * ((buf ^ 1) * npairs + pair) + 1];
        if (sn != 0.0) {
          double vp[RPL], vq[RPL];
#pragma unroll
          for (int r = 0; r < RPL; ++r) {
            vp[r] = Vc[vpa * LD + sub + r * TPP];
            vq[r] = Vc[vpb * LD + sub + r * TPP];
          }
#pragma unroll
          for (int r = 0; r < RPL; ++r) {
            Vc[vpa * LD + sub + r * TPP] = cs * vp[r] - sn * vq[r];
            Vc[vpb * LD + sub + r * TPP] = sn * vp[r] + cs * vq[r];
          }
        }
      }
      if (!isg) {
        vpa = pa;
        vpb = pb;
      }
      buf ^= 1;
      if (ia != 0) pa = pa == m1 ? 1 : pa + 1;
      pb = pb == m1 ? 1 : pb + 1;
      __syncthreads();
    }
    if (!__syncthreads_or(rot)) break;
  }
  if (WITH_V) {
    // the last step's rotations
    if (!isg && live && vpa >= 0) {
      const double cs = rotb[2 * ((buf ^ 1) * npairs + pair)];
      const double sn = rotb[2 * ((buf ^ 1) * npairs + pair) + 1];
      if (sn != 0.0) {
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
          const double vp = Vc[vpa * LD + sub + r * TPP], vq = Vc[vpb * LD + sub + r * TPP];
          Vc[vpa * LD + sub + r * TPP] = cs * vp - sn * vq;
          Vc[vpb * LD + sub + r * TPP] = sn * vp + cs * vq;
        }
      }
    }
    __syncthreads();
  }
  for (int j = tid; j < n; j += nt) {
    double s2 = 0.0;
    for (int i = 0; i < n; ++i) s2 += Gc[j * LD + i] * Gc[j * LD + i];
    sv[j] = sqrt(s2);
  }
  __syncthreads();
  for (int j = tid; j < n; j += nt) {
    int r = 0;
    for (int i = 0; i < n; ++i) r += (sv[i] > sv[j]) || (sv[i] == sv[j] && i < j);
    pos[j] = r;
  }
  __syncthreads();
  for (int idx = tid; idx < n * n; idx += nt) {
    const int j = idx / n, i = idx % n;
    const int pj = pos[j];
    const double sj = sv[j];
    U[(long)i * n + pj] = sj > 0.0 ? Gc[j * LD + i] / sj : (i == pj ? 1.0 : 0.0);
    if (WITH_V) V[(long)i * n + pj] = Vc[j * LD + i];
  }
  for (int j = tid; j < n; j += nt) S[pos[j]] = sv[j];
}

// The same iteration for 64 < n <= 137 on 1024 threads: G in dynamic LDS with a
// padded column stride (n + 1); each column pair of a step is owned by an aligned
// group of lanes (DPP sums).  V is rotated in LDS as well when both fit.  Otherwise
// V lives in ws and the rotations of a sweep are recorded (cs, sn per step and pair)
// and applied to V once per sweep: G is stashed in ws, V brought into the same LDS,
// rotated step by step with the same schedule, written back, and G restored; every
// rotation then costs LDS traffic instead of an L2 round trip per step.
// ws (V_LDS = false): V and the G stash (n (n + 1) doubles each), then
// 2 (n + 1) (n + 1) / 2 doubles of rotations.
constexpr int SVB_NT = 1024;
constexpr size_t SVB_LDS_BYTES = 156 * 1024;

template <bool V_LDS>
__device__ __forceinline__ void jacobi_svd_big_body(int n, const double* G, int ldg, int trans, double* U, double* S, double* V,
                                                    double* ws, double* dyn) {
  __shared__ double sv[SV_MAXN];
  __shared__ int pos[SV_MAXN];
  const int tid = threadIdx.x;
  const int ld = n + 1;
  double* Gc = dyn;
  double* Vc = V_LDS ? dyn + (long)n * ld : ws;
  double* Gs = ws + (long)n * ld;        // G stash while V is in LDS (V_LDS = false)
  double* Rot = ws + 2 * (long)n * ld;   // (cs, sn) per (step, pair) of the current sweep
  for (int idx = tid; idx < n * n; idx += SVB_NT) {
    const int i = idx % n, j = idx / n;
    Gc[j * ld + i] = trans ? G[(long)j * ldg + i] : G[(long)i * ldg + j];
    Vc[j * ld + i] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int npad = n + (n & 1);
  const int npairs = npad / 2;
  int tpp = 1;
  while (tpp * 2 * npairs <= SVB_NT && tpp < 64) tpp *= 2;
  const int pair = tid / tpp, sub = tid % tpp;
  // rows sub, sub + tpp, ...: the lanes of a pair read consecutive rows
  const double eps = n * 2.220446049250313e-16;
  for (int sweep = 0; sweep < 40; ++sweep) {
    int rot = 0;
    for (int step = 0; step < npad - 1; ++step) {
      if (pair < npairs) {
        const int ia = pair, ib = npad - 1 - pair;
        const int pa = ia == 0 ? 0 : 1 + (ia - 1 + step) % (npad - 1);
        const int pb = ib == 0 ? 0 : 1 + (ib - 1 + step) % (npad - 1);
        const int p = pa < pb ? pa : pb, q = pa < pb ? pb : pa;
        double a = 0.0, b = 0.0, cc = 0.0;
        if (q < n) {
          for (int i = sub; i < n; i += tpp) {
            const double gp = Gc[p * ld + i], gq = Gc[q * ld + i];
            a += gp * gp;
            b += gq * gq;
            cc += gp * gq;
          }
        }
        a = group_sum(a, tpp);
        b = group_sum(b, tpp);
        cc = group_sum(cc, tpp);
        double cs = 1.0, sn = 0.0;
        if (q < n && jacobi_rotate(a, b, cc, eps)) {
          jacobi_rotation(a, b, cc, cs, sn);
          for (int i = sub; i < n; i += tpp) {
            const double gp = Gc[p * ld + i], gq = Gc[q * ld + i];
            Gc[p * ld + i] = cs * gp - sn * gq;
            Gc[q * ld + i] = sn * gp + cs * gq;
            if (V_LDS) {
              const double vp = Vc[p * ld + i], vq = Vc[q * ld + i];
              Vc[p * ld + i] = cs * vp - sn * vq;
              Vc[q * ld + i] = sn * vp + cs * vq;
            }
          }
          rot = 1;
        }
        if (!V_LDS && sub == 0) {
          Rot[2 * ((long)step * npairs + pair)] = cs;
          Rot[2 * ((long)step * npairs + pair) + 1] = sn;
        }
      }
      __syncthreads();
    }
    const bool any = __syncthreads_or(rot);
    if (!V_LDS && any) {
      // G out to ws, V into LDS, the sweep's rotations on V, V back, G back
      for (int idx = tid; idx < n * ld; idx += SVB_NT) Gs[idx] = Gc[idx];
      __syncthreads();
      for (int idx = tid; idx < n * ld; idx += SVB_NT) Gc[idx] = Vc[idx];
      __syncthreads();
      for (int step = 0; step < npad - 1; ++step) {
        if (pair < npairs) {
          const int ia = pair, ib = npad - 1 - pair;
          const int pa = ia == 0 ? 0 : 1 + (ia - 1 + step) % (npad - 1);
          const int pb = ib == 0 ? 0 : 1 + (ib - 1 + step) % (npad - 1);
          const int p = pa < pb ? pa : pb, q = pa < pb ? pb : pa;
          const double cs = Rot[2 * ((long)step * npairs + pair)];
          const double sn = Rot[2 * ((long)step * npairs + pair) + 1];
          if (q < n && sn != 0.0) {
            for (int i = sub; i < n; i += tpp) {
              const double vp = Gc[p * ld + i], vq = Gc[q * ld + i];
              Gc[p * ld + i] = cs * vp - sn * vq;
              Gc[q * ld + i] = sn * vp + cs * vq;
            }
          }
        }
        __syncthreads();
      }
      for (int idx = tid; idx < n * ld; idx += SVB_NT) Vc[idx] = Gc[idx];
      __syncthreads();
      for (int idx = tid; idx < n * ld; idx += SVB_NT) Gc[idx] = Gs[idx];
      __syncthreads();
    }
    if (!any) break;
  }
  for (int j = tid; j < n; j += SVB_NT) {
    double s2 = 0.0;
    for (int i = 0; i < n; ++i) s2 += Gc[j * ld + i] * Gc[j * ld + i];
    sv[j] = sqrt(s2);
  }
  __syncthreads();
  for (int j = tid; j < n; j += SVB_NT) {
    int r = 0;
    for (int i = 0; i < n; ++i) r += (sv[i] > sv[j]) || (sv[i] == sv[j] && i < j);
    pos[j] = r;
  }
  __syncthreads();
  for (int idx = tid; idx < n * n; idx += SVB_NT) {
    const int j = idx / n, i = idx % n;
    const int pj = pos[j];
    const double sj = sv[j];
    U[(long)i * n + pj] = sj > 0.0 ? Gc[j * ld + i] / sj : (i == pj ? 1.0 : 0.0);
    V[(long)i * n + pj] = Vc[j * ld + i];
  }
  for (int j = tid; j < n; j += SVB_NT) S[pos[j]] = sv[j];
}

template <int RPL, bool WITH_V>
__global__ __launch_bounds__(SVW_MAX_THREADS) void jacobi_svd_wave_kernel(int n, const double* G, int ldg, int trans,
                                                                          double* U, double* S, double* V) {
  extern __shared__ double dyn[];
  jacobi_svd_wave_body<RPL, WITH_V>(n, G, ldg, trans, U, S, V, dyn);
}

template <bool V_LDS>
__global__ __launch_bounds__(SVB_NT) void jacobi_svd_big_kernel(int n, const double* G, int ldg, int trans, double* U,
                                                               double* S, double* V, double* ws) {
  extern __shared__ double dyn[];
  jacobi_svd_big_body<V_LDS>(n, G, ldg, trans, U, S, V, ws, dyn);
}

// One workgroup per job: the same one-sided Jacobi as the single launches (the jobs
// of one launch share RPL and WITH_V; the block has the threads of the largest).
template <int RPL, bool WITH_V>
__global__ __launch_bounds__(SVW_MAX_THREADS) void jacobi_svd_wave_batch_kernel(SvdBatch b) {
  extern __shared__ double dyn[];
  const SvdJob j = b.job[blockIdx.x];
  jacobi_svd_wave_body<RPL, WITH_V>(j.n, j.G, j.ldg, j.trans, j.U, j.S, j.V, dyn);
}

template <int RPL, bool WITH_V>
static void svw_set_attr() {
  static std::once_flag once;
  std::call_once(once, [] {
    const int bytes = (int)std::max(svw_lds_bytes(SVW_MAXN, 8, true), svw_lds_bytes(SVW_MAXN_LEFT, 16, false));
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&jacobi_svd_wave_kernel<RPL, WITH_V>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&jacobi_svd_wave_batch_kernel<RPL, WITH_V>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  });
}

template <int RPL, bool WITH_V>
static void launch_svw(int n, const double* G, int ldg, int trans, double* U, double* S, double* V, hipStream_t s) {
  svw_set_attr<RPL, WITH_V>();
  hipLaunchKernelGGL((jacobi_svd_wave_kernel<RPL, WITH_V>), dim3(1), dim3(svw_threads(n, WITH_V)),
                     svw_lds_bytes(n, RPL, WITH_V), s, n, G, ldg, trans, U, S, V);
}

template <int RPL, bool WITH_V>
static void launch_svw_batch(const SvdBatch& b, hipStream_t s) {
  svw_set_attr<RPL, WITH_V>();
  int nt = 64;
  size_t lds = 0;
  for (int i = 0; i < b.njob; ++i) {
    nt = std::max(nt, svw_threads(b.job[i].n, WITH_V));
    lds = std::max(lds, svw_lds_bytes(b.job[i].n, RPL, WITH_V));
  }
  hipLaunchKernelGGL((jacobi_svd_wave_batch_kernel<RPL, WITH_V>), dim3(b.njob), dim3(nt), lds, s, b);
}

static void launch_svw_any(int n, const double* G, int ldg, int trans, double* U, double* S, double* V, bool with_v,
                           hipStream_t s) {
  switch (svw_rpl(n) * 2 + (with_v ? 1 : 0)) {
    case 2: launch_svw<1, false>(n, G, ldg, trans, U, S, V, s); break;
    case 3: launch_svw<1, true>(n, G, ldg, trans, U, S, V, s); break;
    case 4: launch_svw<2, false>(n, G, ldg, trans, U, S, V, s); break;
    case 5: launch_svw<2, true>(n, G, ldg, trans, U, S, V, s); break;
    case 8: launch_svw<4, false>(n, G, ldg, trans, U, S, V, s); break;
    case 9: launch_svw<4, true>(n, G, ldg, trans, U, S, V, s); break;
    case 16: launch_svw<8, false>(n, G, ldg, trans, U, S, V, s); break;
    case 17: launch_svw<8, true>(n, G, ldg, trans, U, S, V, s); break;
    case 32: launch_svw<16, false>(n, G, ldg, trans, U, S, V, s); break;
    default: throw Error(TNFEM_EINVAL, "Jacobi SVD: n > 64 with V goes to the 1024-thread kernels");
  }
}

static void launch_svw_batch_any(int rpl, bool with_v, const SvdBatch& b, hipStream_t s) {
  switch (rpl * 2 + (with_v ? 1 : 0)) {
    case 2: launch_svw_batch<1, false>(b, s); break;
    case 3: launch_svw_batch<1, true>(b, s); break;
    case 4: launch_svw_batch<2, false>(b, s); break;
    case 5: launch_svw_batch<2, true>(b, s); break;
    case 8: launch_svw_batch<4, false>(b, s); break;
    case 9: launch_svw_batch<4, true>(b, s); break;
    case 16: launch_svw_batch<8, false>(b, s); break;
    case 17: launch_svw_batch<8, true>(b, s); break;
    case 32: launch_svw_batch<16, false>(b, s); break;
    default: throw Error(TNFEM_EINVAL, "Jacobi SVD batch: n > 64 with V goes to the 1024-thread kernels");
  }
}

template <bool V_LDS>
__global__ __launch_bounds__(SVB_NT) void jacobi_svd_big_batch_kernel(SvdBatch b) {
  extern __shared__ double dyn[];
  const SvdJob j = b.job[blockIdx.x];
  jacobi_svd_big_body<V_LDS>(j.n, j.G, j.ldg, j.trans, j.U, j.S, j.V, j.ws, dyn);
}

void launch_jacobi_svd_batch(const std::vector<SvdJob>& jobs, hipStream_t s) {
  if (jobs.size() > (size_t)SVD_BATCH_MAX) throw Error(TNFEM_EINVAL, "SVD batch: too many jobs");
  static std::once_flag attr_once;
  std::call_once(attr_once, [] {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&jacobi_svd_big_batch_kernel<true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)SVB_LDS_BYTES);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&jacobi_svd_big_batch_kernel<false>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)SVB_LDS_BYTES);
  });
  SvdBatch wave[10], big2, big1;  // wave jobs by (rows per lane, with V)
  size_t m2 = 0, m1 = 0;
  for (const SvdJob& j : jobs) {
    const size_t g = (size_t)j.n * (j.n + 1) * sizeof(double);
    if (j.n <= SVW_MAXN || (j.left_only && j.n <= SVW_MAXN_LEFT)) {
      const int r = svw_rpl(j.n);
      SvdBatch& w = wave[(r == 1 ? 0 : r == 2 ? 1 : r == 4 ? 2 : r == 8 ? 3 : 4) * 2 + (j.left_only ? 0 : 1)];
      w.job[w.njob++] = j;
    } else if (2 * g <= SVB_LDS_BYTES) {
      big2.job[big2.njob++] = j;
      m2 = std::max(m2, 2 * g);
    } else if (g <= SVB_LDS_BYTES) {
      big1.job[big1.njob++] = j;
      m1 = std::max(m1, g);
    } else {
      launch_jacobi_svd(j.n, j.G, j.ldg, j.U, j.S, j.V, j.ws, s, j.trans, j.left_only);
    }
  }
  for (int c = 0; c < 10; ++c) {
    if (!wave[c].njob) continue;
    launch_svw_batch_any(1 << (c / 2), c % 2 == 1, wave[c], s);
    TN_CHECK_LAUNCH();
  }
  if (big2.njob) {
    hipLaunchKernelGGL(jacobi_svd_big_batch_kernel<true>, dim3(big2.njob), dim3(SVB_NT), m2, s, big2);
    TN_CHECK_LAUNCH();
  }
  if (big1.njob) {
    hipLaunchKernelGGL(jacobi_svd_big_batch_kernel<false>, dim3(big1.njob), dim3(SVB_NT), m1, s, big1);
    TN_CHECK_LAUNCH();
  }
}

void launch_jacobi_svd(int n, const double* G, int ldg, double* U, double* S, double* V, double* ws, hipStream_t s,
                       int trans, bool left_only) {
  if (n > SV_MAXN) throw Error(TNFEM_EINVAL, "Jacobi SVD limited to n <= 256");
  if (n <= SVW_MAXN || (left_only && n <= SVW_MAXN_LEFT)) {
    launch_svw_any(n, G, ldg, trans, U, S, V, !left_only, s);
    TN_CHECK_LAUNCH();
    return;
  }
  const size_t gbytes = (size_t)n * (n + 1) * sizeof(double);
  if (gbytes <= SVB_LDS_BYTES) {
    static std::once_flag attr_once;
    std::call_once(attr_once, [] {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&jacobi_svd_big_kernel<true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)SVB_LDS_BYTES);
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&jacobi_svd_big_kernel<false>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)SVB_LDS_BYTES);
    });
    if (2 * gbytes <= SVB_LDS_BYTES)
      hipLaunchKernelGGL(jacobi_svd_big_kernel<true>, dim3(1), dim3(SVB_NT), 2 * gbytes, s, n, G, ldg, trans, U, S, V,
                         ws);
    else
      hipLaunchKernelGGL(jacobi_svd_big_kernel<false>, dim3(1), dim3(SVB_NT), gbytes, s, n, G, ldg, trans, U, S, V,
                         ws);
    TN_CHECK_LAUNCH();
    return;
  }
  hipLaunchKernelGGL(jacobi_svd_kernel, dim3(1), dim3(SV_NT), 0, s, n, G, ldg, trans, U, S, V, ws);
  TN_CHECK_LAUNCH();
}

__global__ void trunc_rank_kernel(int c, const double* S, double tol, int cap, int* out) {
  if (threadIdx.x != 0) return;
  double tot = 0.0;
  for (int j = 0; j < c; ++j) tot += S[j] * S[j];
  double tail = 0.0;
  int r = c;
  for (int j = c - 1; j >= 0; --j) {
    if (tail + S[j] * S[j] <= tol * tol * tot) {
      tail += S[j] * S[j];
      r = j;
    } else {
      break;
    }
  }
  if (r < 1) r = 1;
  if (r > cap) r = cap;
  out[0] = r;
}

void launch_trunc_rank(int c, const double* S, double tol, int cap, int* out, hipStream_t s) {
  hipLaunchKernelGGL(trunc_rank_kernel, dim3(1), dim3(64), 0, s, c, S, tol, cap, out);
  TN_CHECK_LAUNCH();
}

// ----------------------------------------------------------------------------- small helpers

__global__ void copy2d_kernel(int rows, int cols, const double* src, long sld, double* dst, long dld, double alpha,
                              double beta) {
  const long total = (long)rows * cols;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
    const long i = idx / cols, j = idx % cols;
    const double v = alpha * src[i * sld + j];
    dst[i * dld + j] = beta == 0.0 ? v : v + beta * dst[i * dld + j];
  }
}

// dst[i][0 .. c1 + c2) = [src1[i][0 .. c1) | src2[i][0 .. c2)] for rows i (column blocks
// side by side, as the enrichment's augmented basis [U | residual])
__global__ void copy_concat_kernel(int rows, int c1, const double* src1, long ld1, int c2, const double* src2,
                                   long ld2, double* dst, long ldd) {
  const int cols = c1 + c2;
  const long total = (long)rows * cols;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
    const long i = idx / cols;
    const int j = (int)(idx % cols);
    dst[i * ldd + j] = j < c1 ? src1[i * ld1 + j] : src2[i * ld2 + (j - c1)];
  }
}

static int blocks_for(long total) {
  long b = (total + 255) / 256;
  if (b < 1) b = 1;
  if (b > 4096) b = 4096;
  return (int)b;
}

void launch_copy_concat(int rows, int c1, const double* src1, long ld1, int c2, const double* src2, long ld2,
                        double* dst, long ldd, hipStream_t s) {
  if (rows <= 0 || c1 + c2 <= 0 || c1 < 0 || c2 < 0) return;
  hipLaunchKernelGGL(copy_concat_kernel, dim3(blocks_for((long)rows * (c1 + c2))), dim3(256), 0, s, rows, c1, src1,
                     ld1, c2, src2, ld2, dst, ldd);
  TN_CHECK_LAUNCH();
}

void launch_copy2d(int rows, int cols, const double* src, long sld, double* dst, long dld, double alpha, double beta,
                   hipStream_t s) {
  if (rows <= 0 || cols <= 0) return;
  hipLaunchKernelGGL(copy2d_kernel, dim3(blocks_for((long)rows * cols)), dim3(256), 0, s, rows, cols, src, sld, dst,
                     dld, alpha, beta);
  TN_CHECK_LAUNCH();
}

__global__ void scale_vt_kernel(int r, int n, const double* S, const double* V, int ldv, double* W) {
  const long total = (long)r * n;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
    const int i = idx / n, j = idx % n;
    W[idx] = S[i] * V[(long)j * ldv + i];
  }
}

void launch_scale_vt(int r, int n, const double* S, const double* V, int ldv, double* W, hipStream_t s) {
  hipLaunchKernelGGL(scale_vt_kernel, dim3(blocks_for((long)r * n)), dim3(256), 0, s, r, n, S, V, ldv, W);
  TN_CHECK_LAUNCH();
}

__global__ void scale_rows_kernel(int r, int n, const double* S, const double* Vt, int ldv, double* W) {
  const long total = (long)r * n;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
    const int i = idx / n, j = idx % n;
    W[idx] = S[i] * Vt[(long)i * ldv + j];
  }
}

void launch_scale_rows(int r, int n, const double* S, const double* Vt, int ldv, double* W, hipStream_t s) {
  hipLaunchKernelGGL(scale_rows_kernel, dim3(blocks_for((long)r * n)), dim3(256), 0, s, r, n, S, Vt, ldv, W);
  TN_CHECK_LAUNCH();
}

__global__ void core_transpose_kernel(int ra, int n, int rb, const double* in, double* out) {
  const long total = (long)ra * n * rb;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
    const int b = idx % rb;
    const int i = (idx / rb) % n;
    const int a = idx / ((long)rb * n);
    out[((long)b * n + i) * ra + a] = in[idx];
  }
}

void launch_core_transpose(int ra, int n, int rb, const double* in, double* out, hipStream_t s) {
  hipLaunchKernelGGL(core_transpose_kernel, dim3(blocks_for((long)ra * n * rb)), dim3(256), 0, s, ra, n, rb, in, out);
  TN_CHECK_LAUNCH();
}

// Several core transposes in one launch: job j covers flattened blocks beg[j] ..
// beg[j + 1] - 1, 256 elements each.
__global__ __launch_bounds__(256) void core_transpose_multi_kernel(TransposeJobs J) {
  int j = 0;
  while (j + 1 < J.n && (int)blockIdx.x >= J.beg[j + 1]) ++j;
  const TransposeJob& t = J.job[j];
  const long idx = (long)(blockIdx.x - J.beg[j]) * 256 + threadIdx.x;
  const long total = (long)t.ra * t.n * t.rb;
  if (idx >= total) return;
  const int b = idx % t.rb;
  const int i = (idx / t.rb) % t.n;
  const int a = idx / ((long)t.rb * t.n);
  t.out[((long)b * t.n + i) * t.ra + a] = t.in[idx];
}

void launch_core_transpose_multi(const TransposeJob* jobs, int n, hipStream_t s) {
  for (int off = 0; off < n; off += TRANSPOSE_MULTI_MAX) {
    TransposeJobs J{};
    J.n = std::min(TRANSPOSE_MULTI_MAX, n - off);
    long blocks = 0;
    for (int j = 0; j < J.n; ++j) {
      J.job[j] = jobs[off + j];
      J.beg[j] = (int)blocks;
      blocks += ((long)jobs[off + j].ra * jobs[off + j].n * jobs[off + j].rb + 255) / 256;
    }
    J.beg[J.n] = (int)blocks;
    if (blocks == 0) continue;
    if (blocks > INT32_MAX / 2) throw Error(TNFEM_EINVAL, "core transpose launch too large");
    hipLaunchKernelGGL(core_transpose_multi_kernel, dim3((unsigned)blocks), dim3(256), 0, s, J);
    TN_CHECK_LAUNCH();
  }
}

__global__ void sub_kernel(long n, const double* a, const double* b, double* out) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    out[i] = a[i] - b[i];
}

void launch_sub(long n, const double* a, const double* b, double* out, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(sub_kernel, dim3(blocks_for(n)), dim3(256), 0, s, n, a, b, out);
  TN_CHECK_LAUNCH();
}

__global__ void nan_check_kernel(long n, const double* x, int* flag) {
  int bad = 0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    bad |= !isfinite(x[i]);
  if (bad) atomicOr(flag, 1);
}

void launch_nan_check(long n, const double* x, int* flag, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(nan_check_kernel, dim3(blocks_for(n)), dim3(256), 0, s, n, x, flag);
  TN_CHECK_LAUNCH();
}

}  // namespace tnfem

// ----------------------------------------------------------------------------- thin SVD

namespace tnfem {

// Workspace: the input in tall orientation, Q, R, the Jacobi factors and the larger of the
// QR's and the Jacobi kernel's own workspace.
size_t svd_ws_doubles(int m, int n) {
  const int mm = std::max(m, n), nn = std::min(m, n);
  return (size_t)mm * nn * 2 + (size_t)nn * nn * 3 +
         std::max(qr_ws_doubles(mm, nn), (size_t)nn * nn * 3 + 3 * nn) + 8;
}

void svd_device(int m, int n, const double* A, double* U, double* S, double* Vt, double* ws, size_t ws_cap,
                hipStream_t st) {
  const bool tall = m >= n;
  const int mm = tall ? m : n, nn = tall ? n : m;  // work on the tall orientation
  if (ws_cap < svd_ws_doubles(m, n)) throw Error(TNFEM_EINVAL, "SVD workspace too small");
  double* At = ws;                       // mm x nn (transposed input when wide)
  double* Q = At + (size_t)mm * nn;      // mm x nn
  double* R = Q + (size_t)mm * nn;       // nn x nn
  double* UR = R + (size_t)nn * nn;      // nn x nn
  double* V = UR + (size_t)nn * nn;      // nn x nn
  double* qws = V + (size_t)nn * nn;     // QR workspace, then the Jacobi kernel's
  const double* src = A;
  if (!tall) {
    launch_core_transpose(m, 1, n, A, At, st);  // At = A^T (n x m)
    src = At;
  }
  const size_t qws_cap = ws_cap - (size_t)(qws - ws);
  launch_qr(mm, nn, src, nn, Q, nn, R, nn, qws, qws_cap, st);
  launch_jacobi_svd(nn, R, nn, V, S, UR, qws, st, 1);  // on R^T: outputs swapped
  GemmDesc g;
  if (tall) {
    // U = Q UR (m x n); Vt = V^T
    g.A = Q; g.a_sm = nn; g.a_sk = 1;
    g.B = UR; g.b_sk = nn; g.b_sn = 1;
    g.C = U; g.c_sm = nn; g.c_sn = 1;
    g.M = mm; g.N = nn; g.K = nn;
    launch_gemm(g, st);
    launch_core_transpose(nn, 1, nn, V, Vt, st);
  } else {
    // A^T = (Q UR) S V^T  =>  A = V S (Q UR)^T: U = V (m x m), Vt = (Q UR)^T (m x n)
    launch_copy2d(nn, nn, V, nn, U, nn, 1.0, 0.0, st);
    g.A = UR; g.a_sm = 1; g.a_sk = nn;   // UR^T
    g.B = Q; g.b_sk = 1; g.b_sn = nn;    // Q^T
    g.C = Vt; g.c_sm = mm; g.c_sn = 1;
    g.M = nn; g.N = mm; g.K = nn;
    launch_gemm(g, st);
  }
}

}  // namespace tnfem
