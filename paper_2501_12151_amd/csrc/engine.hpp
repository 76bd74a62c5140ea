// Device-resident AMEn engine: problem state, contraction plans, the sweep.
#pragma once

#include <hip/hip_runtime.h>

#include <memory>
#include <vector>

#include "assembly.hpp"
#include "kernels.hpp"

namespace tnfem {

void hip_check(hipError_t e, const char* what);

// Caller-supplied device allocator (e.g. bound to torch's caching allocator); alloc == NULL
// means hipMalloc / hipFree.
struct DeviceAllocator {
  tnfem_alloc_fn alloc = nullptr;
  tnfem_free_fn free = nullptr;
  void* user = nullptr;
  hipStream_t stream = nullptr;
  void* allocate(size_t bytes) const;
  void release(void* p) const;
};

// Owner of device allocations made for one object; freed on destruction.
class DevArena {
 public:
  // dry = true: allocations are only counted (null pointers, no copies), for
  // sizing a problem's device memory before anything is allocated
  explicit DevArena(bool dry = false) : dry_(dry) {}
  ~DevArena();
  void set_allocator(const DeviceAllocator* a) { alloc_ = a; }
  void* alloc(size_t bytes);
  template <class T>
  T* upload(const std::vector<T>& v, hipStream_t s);
  void release_all();
  size_t bytes() const { return bytes_; }

 private:
  std::vector<void*> ptrs_;
  size_t bytes_ = 0;
  bool dry_ = false;
  const DeviceAllocator* alloc_ = nullptr;
};

// Contraction plan of one operator core in one chain orientation.
// Stage 1: T1[slot] = L[:, b_slot, :] x[:, i_slot, :] for every used (b, i).
// Stage 2 (dense plans only): T2[(io, e)] = sum_slot A2[slot][(io, e)] T1[slot].
// Stage 3: apply terms (grouped by io): y[:, io, :] += v T[a] Rt[:, e = b, :]^T;
//          interface terms (grouped by e): Lnew[:, e, :] += v W[:, io = a, :]^T T[b].
struct Plan {
  int Rl = 1, Rr = 1, n = 1;
  int nslot = 0;
  bool dense = false;
  int *slot_beg = nullptr, *slot_b = nullptr, *slot_i = nullptr;
  double* A2 = nullptr;
  int *ap_beg = nullptr, *ap_a = nullptr, *ap_b = nullptr;
  double* ap_v = nullptr;
  int n_ap = 0, ap_max = 1;
  int *en_beg = nullptr, *en_a = nullptr, *en_b = nullptr;
  double* en_v = nullptr;
  int n_en = 0, en_max = 1;
  // all nonzero terms grouped by (out, in) mode pair (j n + i): (b, e, v)
  int *bk_beg = nullptr, *bk_b = nullptr, *bk_e = nullptr;
  double* bk_v = nullptr;
  // Term lists of the nonzeros (for dense plans: the alternative evaluation by
  // the fused kernel, cheaper when the ranks next to this core are small).
  int sp_nslot = 0, sp_n_ap = 0, sp_ap_max = 1;
  int *sp_slot_b = nullptr, *sp_slot_i = nullptr, *sp_ap_beg = nullptr, *sp_ap_a = nullptr, *sp_ap_b = nullptr;
  double* sp_ap_v = nullptr;
  int* sp_ap_c = nullptr;        // per term: b * 16 + i of its slot
  std::vector<int> sp_beg_h;     // host copy of sp_ap_beg (n + 1 offsets)
  int n_t1() const { return nslot; }
  int n_t2() const { return dense ? n * Rr : 0; }
};

struct Context {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  DeviceAllocator allocator;  // device memory of the context's problems and scratch
  DevArena arena;
  double* scratch = nullptr;  // for primitives
  size_t scratch_doubles = 0;
  double* splitk = nullptr;   // split-K partial tiles for primitives
  size_t splitk_cap = 0;
  double* ensure_scratch(size_t doubles);
  void ensure_splitk();
};

struct Problem;

// Buffers of the outer iterative refinement (allocated on first use): the refined solution
// u (K cores), the interfaces between the iterate and u through A (X-A-u, Z-A-u; K + 1 bonds
// each), the cores of u + d before rounding, and the thin-SVD scratch of the rounding.
struct IrBuffers {
  int cap = 0, rho = 0;
  DevArena arena;
  std::vector<double*> U, EuA, EzuA, Sum;
  double *uspare = nullptr, *t1 = nullptr, *t2 = nullptr, *su = nullptr, *ss = nullptr, *svt = nullptr,
         *svdws = nullptr;
  size_t sum_cap = 0, svdws_cap = 0;
};

// Workspace of one problem for a given rank cap.
struct Workspace {
  int cap = 0, rho = 0;
  DevArena arena;
  std::vector<double*> X, Z;  // K core buffers each (+1 spare for swaps)
  double *Xspare = nullptr, *Zspare = nullptr;
  // second core sets: a change of orientation transposes every core into them at once
  std::vector<double*> Xalt, Zalt;
  std::vector<double*> EA, Eb, EzA, Ezb;  // K + 1 bond buffers
  double *T1 = nullptr, *T2 = nullptr;
  // the Z interface update's own stage products, so that it runs beside the X one
  double *T1z = nullptr, *T2z = nullptr, *Tbz = nullptr;
  double *g = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *w = nullptr;
  double* binv = nullptr;  // inverses of the diagonal mode blocks of the local operator
  double *Tb = nullptr, *gz = nullptr, *yz = nullptr, *ge = nullptr, *ye = nullptr;
  double *Qx = nullptr, *Rx = nullptr, *UR = nullptr, *S = nullptr, *V = nullptr, *Ur = nullptr, *SVt = nullptr,
         *xt = nullptr, *aug = nullptr, *xT = nullptr, *Qa = nullptr, *Ra = nullptr, *Wm = nullptr, *qrws = nullptr;
  double *Rz = nullptr, *qrwsz = nullptr;  // R and scratch of the residual-TT QR
  size_t qrws_cap = 0, qrwsz_cap = 0;     // doubles at qrws and qrwsz
  double *scal = nullptr, *part = nullptr;
  double* splitk = nullptr;
  size_t splitk_cap = 0;
  double* fpart = nullptr;  // fused-apply partial tiles
  size_t fpart_cap = 0;
  double* stage = nullptr;  // slot products of the fused apply at ranks above 64
  size_t stage_bytes = 0;
  double *Bloc = nullptr, *Mloc = nullptr;  // explicit local matrix (dense plans, small local systems)
  size_t bloc_n = 0, mloc_cap = 0;
  int* flag = nullptr;
  int* drank = nullptr;
  void* host_pinned = nullptr;
  size_t bytes = 0;
  std::unique_ptr<GemmProfile> profile;
  std::unique_ptr<IrBuffers> ir;  // outer refinement (allocated on first use)
  ~Workspace() {
    if (host_pinned) (void)hipHostFree(host_pinned);
  }
};

struct Problem {
  Context* ctx = nullptr;
  Assembled host;
  int K = 0;
  std::vector<int> modes;
  std::vector<Plan> plans[2];
  std::vector<double*> bcore[2];
  std::vector<int> brank[2];  // K + 1
  std::vector<int> mrank[2];  // K + 1
  int Rmax = 1, smax = 1, maxn = 1;
  size_t t1max_slots = 1, t2max_slots = 1;
  size_t sp_slots_max = 1;  // most slots of a sparse plan (stage of the two-stage fused apply)
  DevArena arena;
  size_t device_bytes = 0;  // bytes the operator plans and load cores take on the device
  bool uploaded = false;
  std::unique_ptr<Workspace> ws;
  void ensure_workspace(int cap, int rho);
  size_t workspace_bytes(int cap, int rho) const;  // device bytes ensure_workspace would allocate
  void ensure_ir(int cap, int rho);                 // refinement buffers (after ensure_workspace)
};

// Host TT object.
struct HostTT {
  std::vector<int> modes, ranks;
  std::vector<std::vector<double>> cores;
};

// Host assembly and contraction plans, sized but not uploaded (device_bytes set).
std::unique_ptr<Problem> make_problem_host(const tnfem_problem_desc& desc);
// Uploads the plans and load cores of a host-built problem to ctx's device.
void upload_problem(Context* ctx, Problem& P);
// Both steps.
std::unique_ptr<Problem> make_problem(Context* ctx, const tnfem_problem_desc& desc);

// Contractions on the problem's plans (device pointers, asynchronous on s).
struct Flops {
  double total = 0;
};
void dev_local_apply(Problem& P, const Plan& pl, int p, int q, int s, int t, const double* L, const double* x,
                     const double* Rt, double* y, const int* skip, hipStream_t st, Flops* f);
void dev_local_apply_fused(Problem& P, const Plan& pl, int p, int q, int s, int t, const double* L, const double* x,
                           const double* Rt, double* y, int precision, hipStream_t st);
void dev_env_update(Problem& P, const Plan& pl, int p, int q, int s, int t, const double* W, const double* L,
                    const double* X, double* Lnew, hipStream_t st, Flops* f);

int run_solve(Problem& P, const tnfem_solve_opts& o, HostTT& out, tnfem_solve_stats& st);
// Lockstep solve of several problems of the same dimension and level in one context
// (FP64): per problem the same steps and results as run_solve, with the CG iterations
// of all problems issued as shared launches.  Per-problem status in rcs.
int run_solve_batch(std::vector<Problem*>& Ps, const tnfem_solve_opts& o, std::vector<HostTT>& outs,
                    std::vector<tnfem_solve_stats>& stats, std::vector<int>& rcs);

}  // namespace tnfem

// Host TT handed out through the C ABI.
struct tnfem_tt {
  tnfem::HostTT t;
};
