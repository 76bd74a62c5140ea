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
#include <hip/hip_runtime.h>

#include <cfloat>
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

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over a group of `width` consecutive lanes (width a power of two <= 64).
__device__ inline double group_sum(double v, int width) {
  for (int off = width >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
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
  int tiles_n;
};

constexpr int BK = 16;

// 4 waves in a 2 x 2 arrangement; each wave owns WMB x WNB blocks of 16 x 16.
template <int WMB, int WNB>
__global__ __launch_bounds__(256) void gemm_grouped_kernel(GemmArgs g) {
  constexpr int TM = 32 * WMB, TN = 32 * WNB;
  __shared__ double sA[BK][TM + 1];
  __shared__ double sB[BK][TN + 1];
  if (g.skip && *g.skip) return;
  const int grp = blockIdx.y;
  const int tile = blockIdx.x;
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
  d4_t acc[WMB][WNB];
  for (int i = 0; i < WMB; ++i)
    for (int j = 0; j < WNB; ++j) acc[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};

  const bool a_kfast = (g.a_sk == 1);
  const bool b_nfast = (g.b_sn == 1);
  for (int t = tb; t < te; ++t) {
    const int ai = g.grp_beg ? g.t_a[t] : t;
    const int bi = g.grp_beg ? g.t_b[t] : t;
    const double v = g.t_v ? g.t_v[t] : 1.0;
    const double* Ab = g.A + (long)ai * g.a_slot;
    const double* Bb = g.B + (long)bi * g.b_slot;
    for (int k0 = 0; k0 < g.K; k0 += BK) {
      // stage A tile (TM x BK) k-major
      for (int idx = tid; idx < TM * BK; idx += 256) {
        int mm, kk;
        if (a_kfast) { mm = idx / BK; kk = idx % BK; }
        else { mm = idx % TM; kk = idx / TM; }
        const int gm = m0 + mm, gk = k0 + kk;
        sA[kk][mm] = (gm < g.M && gk < g.K) ? v * Ab[(long)gm * g.a_sm + (long)gk * g.a_sk] : 0.0;
      }
      for (int idx = tid; idx < TN * BK; idx += 256) {
        int nn, kk;
        if (b_nfast) { nn = idx % TN; kk = idx / TN; }
        else { nn = idx / BK; kk = idx % BK; }
        const int gn = n0 + nn, gk = k0 + kk;
        sB[kk][nn] = (gn < g.N && gk < g.K) ? Bb[(long)gk * g.b_sk + (long)gn * g.b_sn] : 0.0;
      }
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
  }
  const int ci = g.grp_c ? g.grp_c[grp] : grp;
  double* Cb = g.C + (long)ci * g.c_slot;
  for (int i = 0; i < WMB; ++i)
    for (int j = 0; j < WNB; ++j) {
      const int col = n0 + wn * 16 * WNB + j * 16 + lrow;
      for (int q = 0; q < 4; ++q) {
        // v_mfma_f64_16x16x4f64 result: D[r][c] is in lane c + 16 (r % 4), register r / 4
        const int row = m0 + wm * 16 * WMB + i * 16 + 4 * q + lk;
        if (row < g.M && col < g.N) {
          double* c = Cb + (long)row * g.c_sm + (long)col * g.c_sn;
          const double val = g.alpha * acc[i][j][q];
          *c = (g.beta == 0.0) ? val : val + g.beta * *c;
        }
      }
    }
}

static thread_local GemmProfile* g_prof = nullptr;
void set_gemm_profile(GemmProfile* p) { g_prof = p; }

GemmProfile::~GemmProfile() {
  for (hipEvent_t e : ev) (void)hipEventDestroy(e);
}

double GemmProfile::total_ms(double* total_flops) {
  double ms = 0.0, fl = 0.0;
  if (used > 0) (void)hipEventSynchronize(ev[2 * used - 1]);
  for (size_t i = 0; i < used; ++i) {
    float t = 0.0f;
    if (hipEventElapsedTime(&t, ev[2 * i], ev[2 * i + 1]) == hipSuccess) ms += t;
    fl += flops[i];
  }
  if (total_flops) *total_flops = fl;
  return ms;
}

static void launch_gemm_impl(const GemmDesc& d, hipStream_t s);

void launch_gemm(const GemmDesc& d, hipStream_t s) {
  if (d.M <= 0 || d.N <= 0 || d.ngroups <= 0) return;
  GemmProfile* p = g_prof;
  if (p && p->used < p->limit) {
    while (p->ev.size() < 2 * (p->used + 1)) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) throw Error(TNFEM_EDEVICE, "hipEventCreate");
      p->ev.push_back(e);
    }
    hipEvent_t a = p->ev[2 * p->used], b = p->ev[2 * p->used + 1];
    (void)hipEventRecord(a, s);
    launch_gemm_impl(d, s);
    (void)hipEventRecord(b, s);
    p->flops.push_back(d.flops);
    p->used++;
    return;
  }
  launch_gemm_impl(d, s);
}

static void launch_gemm_impl(const GemmDesc& d, hipStream_t s) {
  GemmArgs a{d.A, d.a_slot, d.a_sm, d.a_sk, d.B, d.b_slot, d.b_sk, d.b_sn, d.C, d.c_slot, d.c_sm, d.c_sn,
             d.M, d.N, d.K, d.grp_beg, d.grp_c, d.t_a, d.t_b, d.t_v, d.alpha, d.beta, d.skip, 0};
  if (d.M >= 64 && d.N >= 64) {
    a.tiles_n = (d.N + 63) / 64;
    dim3 grid(((d.M + 63) / 64) * a.tiles_n, d.ngroups);
    hipLaunchKernelGGL((gemm_grouped_kernel<2, 2>), grid, dim3(256), 0, s, a);
  } else {
    a.tiles_n = (d.N + 31) / 32;
    dim3 grid(((d.M + 31) / 32) * a.tiles_n, d.ngroups);
    hipLaunchKernelGGL((gemm_grouped_kernel<1, 1>), grid, dim3(256), 0, s, a);
  }
  TN_CHECK_LAUNCH();
}

// ----------------------------------------------------------------------------- CG

constexpr int CG_NT = 256;
constexpr int CG_MAXB = 512;

static int cg_blocks(int n) {
  int b = (n + CG_NT * 4 - 1) / (CG_NT * 4);
  return b < 1 ? 1 : (b > CG_MAXB ? CG_MAXB : b);
}

// Last-block reduction of NV partial sums per block.  Returns true in the last block,
// with out[] holding the totals (valid in every thread of that block).
template <int NV>
__device__ bool last_block_reduce(const double (&mine)[NV], double* part, int* counter, double* out) {
  __shared__ double red[CG_NT / 64];
  __shared__ bool am_last;
  double tot[NV];
  for (int v = 0; v < NV; ++v) tot[v] = block_sum<CG_NT>(mine[v], red);
  if (threadIdx.x == 0) {
    for (int v = 0; v < NV; ++v) part[v * CG_MAXB + blockIdx.x] = tot[v];
    __threadfence();
    const int prev = atomicAdd(counter, 1);
    am_last = (prev == (int)gridDim.x - 1);
  }
  __syncthreads();
  if (!am_last) return false;
  __threadfence();
  for (int v = 0; v < NV; ++v) {
    double s = 0.0;
    for (int b = threadIdx.x; b < (int)gridDim.x; b += CG_NT) s += __builtin_nontemporal_load(&part[v * CG_MAXB + b]);
    out[v] = block_sum<CG_NT>(s, red);
  }
  return true;
}

__global__ __launch_bounds__(CG_NT) void cg_init_kernel(int n, const double* g, const double* q, const double* dinv,
                                                        double* r, double* z, double* p, double* scal, int* flag,
                                                        double* part, double tol, int maxit) {
  double loc[3] = {0.0, 0.0, 0.0};  // rz, rr, gg
  for (int i = blockIdx.x * CG_NT + threadIdx.x; i < n; i += gridDim.x * CG_NT) {
    const double gi = g[i];
    const double ri = gi - q[i];
    const double zi = ri * dinv[i];
    r[i] = ri;
    z[i] = zi;
    p[i] = zi;
    loc[0] += ri * zi;
    loc[1] += ri * ri;
    loc[2] += gi * gi;
  }
  double tot[3];
  if (last_block_reduce<3>(loc, part, &flag[CG_COUNTER], tot) && threadIdx.x == 0) {
    const double rr = tot[1], gg = tot[2];
    const double gn = sqrt(gg);
    const double res = gg > 0.0 ? sqrt(rr) / gn : (rr == 0.0 ? 0.0 : 1.0);
    const double thr = fmax(0.1 * res, 0.5 * tol) * gn;
    scal[CG_RZ] = tot[0];
    scal[CG_RR] = rr;
    scal[CG_GG] = gg;
    scal[CG_RES] = res;
    scal[CG_THR2] = thr * thr;
    flag[CG_ITERS] = 0;
    flag[CG_MAXIT] = maxit;
    flag[CG_DONE] = (res <= 0.5 * tol || maxit <= 0) ? 1 : 0;
    flag[CG_COUNTER] = 0;
  }
}

__global__ __launch_bounds__(CG_NT) void cg_dot_kernel(int n, const double* p, const double* q, double* scal,
                                                       int* flag, double* part) {
  if (flag[CG_DONE]) return;
  double loc[1] = {0.0};
  for (int i = blockIdx.x * CG_NT + threadIdx.x; i < n; i += gridDim.x * CG_NT) loc[0] += p[i] * q[i];
  double tot[1];
  if (last_block_reduce<1>(loc, part, &flag[CG_COUNTER], tot) && threadIdx.x == 0) {
    scal[CG_PQ] = tot[0];
    flag[CG_COUNTER] = 0;
  }
}

__global__ __launch_bounds__(CG_NT) void cg_update_kernel(int n, double* x, const double* p, const double* q, double* r,
                                                          double* z, const double* dinv, double* scal, int* flag,
                                                          double* part) {
  if (flag[CG_DONE]) return;
  const double pq = scal[CG_PQ];
  if (!(pq > 0.0)) {  // breakdown: stop without updating (every block takes this branch)
    if (blockIdx.x == 0 && threadIdx.x == 0) flag[CG_DONE] = 2;
    return;
  }
  const double alpha = scal[CG_RZ] / pq;
  double loc[2] = {0.0, 0.0};  // rz, rr
  for (int i = blockIdx.x * CG_NT + threadIdx.x; i < n; i += gridDim.x * CG_NT) {
    x[i] += alpha * p[i];
    const double ri = r[i] - alpha * q[i];
    const double zi = ri * dinv[i];
    r[i] = ri;
    z[i] = zi;
    loc[0] += ri * zi;
    loc[1] += ri * ri;
  }
  double tot[2];
  if (last_block_reduce<2>(loc, part, &flag[CG_COUNTER], tot) && threadIdx.x == 0) {
    scal[CG_BETA] = tot[0] / scal[CG_RZ];
    scal[CG_RZ] = tot[0];
    scal[CG_RR] = tot[1];
    const int it = flag[CG_ITERS] + 1;
    flag[CG_ITERS] = it;
    if (tot[1] <= scal[CG_THR2] || it >= flag[CG_MAXIT]) flag[CG_DONE] = 1;
    flag[CG_COUNTER] = 0;
  }
}

__global__ __launch_bounds__(CG_NT) void cg_pupdate_kernel(int n, double* p, const double* z, const double* scal,
                                                           const int* flag) {
  if (flag[CG_DONE]) return;
  const double beta = scal[CG_BETA];
  for (int i = blockIdx.x * CG_NT + threadIdx.x; i < n; i += gridDim.x * CG_NT) p[i] = z[i] + beta * p[i];
}

void launch_cg_init(int n, const double* g, const double* q, const double* dinv, double* r, double* z, double* p,
                    double* scal, int* flag, double* part, double tol, int maxit, hipStream_t s) {
  hipLaunchKernelGGL(cg_init_kernel, dim3(cg_blocks(n)), dim3(CG_NT), 0, s, n, g, q, dinv, r, z, p, scal, flag, part,
                     tol, maxit);
  TN_CHECK_LAUNCH();
}
void launch_cg_dot(int n, const double* p, const double* q, double* scal, int* flag, double* part, hipStream_t s) {
  hipLaunchKernelGGL(cg_dot_kernel, dim3(cg_blocks(n)), dim3(CG_NT), 0, s, n, p, q, scal, flag, part);
  TN_CHECK_LAUNCH();
}
void launch_cg_update(int n, double* x, const double* p, const double* q, double* r, double* z, const double* dinv,
                      double* scal, int* flag, double* part, hipStream_t s) {
  hipLaunchKernelGGL(cg_update_kernel, dim3(cg_blocks(n)), dim3(CG_NT), 0, s, n, x, p, q, r, z, dinv, scal, flag,
                     part);
  TN_CHECK_LAUNCH();
}
void launch_cg_pupdate(int n, double* p, const double* z, const double* scal, const int* flag, hipStream_t s) {
  hipLaunchKernelGGL(cg_pupdate_kernel, dim3(cg_blocks(n)), dim3(CG_NT), 0, s, n, p, z, scal, flag);
  TN_CHECK_LAUNCH();
}

// ----------------------------------------------------------------------------- local diagonal

__global__ void local_diag_kernel(int p, int n, int t, int Rl, int Rr, const double* L, const double* Rt,
                                  const int* dg_beg, const int* dg_b, const int* dg_e, const double* dg_v,
                                  double* dinv) {
  const long total = (long)p * n * t;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
    const int c = idx % t;
    const int i = (idx / t) % n;
    const int a = idx / ((long)t * n);
    double s = 0.0;
    for (int k = dg_beg[i]; k < dg_beg[i + 1]; ++k) {
      const double lv = L[((long)a * Rl + dg_b[k]) * p + a];
      const double rv = Rt[((long)c * Rr + dg_e[k]) * t + c];
      s += dg_v[k] * lv * rv;
    }
    dinv[idx] = s > 0.0 ? 1.0 / s : 1.0;
  }
}

void launch_local_diag(int p, int n, int t, int Rl, int Rr, const double* L, const double* Rt, const int* dg_beg,
                       const int* dg_b, const int* dg_e, const double* dg_v, double* dinv, hipStream_t s) {
  const long total = (long)p * n * t;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(local_diag_kernel, dim3(blocks), dim3(256), 0, s, p, n, t, Rl, Rr, L, Rt, dg_beg, dg_b, dg_e,
                     dg_v, dinv);
  TN_CHECK_LAUNCH();
}

// ----------------------------------------------------------------------------- QR

constexpr int QR_NT = 256;

__global__ __launch_bounds__(QR_NT) void qr_kernel(int m, int n, const double* A, int lda, double* Q, int ldq,
                                                   double* R, int ldr, double* ws) {
  __shared__ double red[QR_NT / 64];
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int c = m < n ? m : n;
  double* W = ws;                  // m x n, column-major
  double* Qc = ws + (long)m * n;   // m x c, column-major
  double* tau = Qc + (long)m * c;  // c
  double* diag = tau + c;          // c
  for (long idx = tid; idx < (long)m * n; idx += QR_NT) {
    const int i = idx / n, j = idx % n;
    W[(long)j * m + i] = A[(long)i * lda + j];
  }
  __syncthreads();
  for (int j = 0; j < c; ++j) {
    double* v = W + (long)j * m;
    double loc = 0.0;
    for (int i = j + tid; i < m; i += QR_NT) loc += v[i] * v[i];
    const double s = block_sum<QR_NT>(loc, red);
    const double x0 = v[j];
    const double nrm = sqrt(s);
    double tj = 0.0, alpha = 0.0, v0 = x0;
    if (nrm > 0.0) {
      alpha = x0 >= 0.0 ? -nrm : nrm;
      v0 = x0 - alpha;
      tj = 2.0 / (s - x0 * x0 + v0 * v0);
    }
    __syncthreads();
    if (tid == 0) {
      v[j] = v0;
      tau[j] = tj;
      diag[j] = alpha;
    }
    __syncthreads();
    if (tj != 0.0) {
      for (int col = j + 1 + wave; col < n; col += QR_NT / 64) {
        double* w = W + (long)col * m;
        double part = 0.0;
        for (int i = j + lane; i < m; i += 64) part += v[i] * w[i];
        const double f = tj * wave_sum(part);
        for (int i = j + lane; i < m; i += 64) w[i] -= f * v[i];
      }
    }
    __syncthreads();
  }
  for (long idx = tid; idx < (long)c * n; idx += QR_NT) {
    const int i = idx / n, jj = idx % n;
    R[(long)i * ldr + jj] = jj < i ? 0.0 : (jj == i ? diag[i] : W[(long)jj * m + i]);
  }
  for (long idx = tid; idx < (long)m * c; idx += QR_NT) {
    const int jj = idx / m, i = idx % m;
    Qc[idx] = (i == jj) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int j = c - 1; j >= 0; --j) {
    const double tj = tau[j];
    if (tj != 0.0) {
      const double* v = W + (long)j * m;
      for (int col = j + wave; col < c; col += QR_NT / 64) {
        double* q = Qc + (long)col * m;
        double part = 0.0;
        for (int i = j + lane; i < m; i += 64) part += v[i] * q[i];
        const double f = tj * wave_sum(part);
        for (int i = j + lane; i < m; i += 64) q[i] -= f * v[i];
      }
    }
    __syncthreads();
  }
  for (long idx = tid; idx < (long)m * c; idx += QR_NT) {
    const int i = idx / c, jj = idx % c;
    Q[(long)i * ldq + jj] = Qc[(long)jj * m + i];
  }
}

void launch_qr(int m, int n, const double* A, int lda, double* Q, int ldq, double* R, int ldr, double* ws,
               hipStream_t s) {
  hipLaunchKernelGGL(qr_kernel, dim3(1), dim3(QR_NT), 0, s, m, n, A, lda, Q, ldq, R, ldr, ws);
  TN_CHECK_LAUNCH();
}

// ----------------------------------------------------------------------------- Jacobi SVD

constexpr int SV_NT = 256;
constexpr int SV_LDS_MAXN = 64;
constexpr int SV_MAXN = 256;

__global__ __launch_bounds__(SV_NT) void jacobi_svd_kernel(int n, const double* G, int ldg, double* U, double* S,
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
    Gc[idx] = G[(long)i * ldg + j];
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
  const double eps = 1e-15;
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
        if (q < n && cc != 0.0 && fabs(cc) > eps * sqrt(a * b)) {
          const double zeta = (b - a) / (2.0 * cc);
          const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = cs * tt;
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

void launch_jacobi_svd(int n, const double* G, int ldg, double* U, double* S, double* V, double* ws, hipStream_t s) {
  if (n > SV_MAXN) throw Error(TNFEM_EINVAL, "Jacobi SVD limited to n <= 256");
  hipLaunchKernelGGL(jacobi_svd_kernel, dim3(1), dim3(SV_NT), 0, s, n, G, ldg, U, S, V, ws);
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

static int blocks_for(long total) {
  long b = (total + 255) / 256;
  if (b < 1) b = 1;
  if (b > 4096) b = 4096;
  return (int)b;
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
