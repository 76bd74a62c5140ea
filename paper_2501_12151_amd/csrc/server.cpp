// Continuous-batching request server: elasticity solves of different sizes,
// materials and loads share one GPU.
//
// A request is queued at submission.  Each worker slot owns a HIP stream (one
// context); a free slot takes the oldest queued request together with the
// queued requests of the same shape bucket (same dimension, level and solve
// options, no outer refinement; up to max_batch of them), assembles their problems on the host,
// computes the device bytes their solves will hold (operator plans, load cores and
// workspace) and uploads them once that fits in the HBM budget next to the
// requests already running (nothing is allocated on the device before admission).  A bucket of several requests is solved in lockstep with shared
// launches of the local CG iterations (run_solve_batch); different slots run
// on different streams, so their work overlaps on the device.  A request's
// arithmetic does not depend on what else runs (per-request kernels and
// reductions), so every result equals the request solved alone.  Latency is
// measured from submission to the request's own completion.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "common.hpp"
#include "assembly.hpp"
#include "engine.hpp"

namespace tnfem {

struct Request {
  long long id = 0;
  tnfem_problem_desc desc{};
  std::vector<double> layer;
  std::vector<double> ew;
  std::vector<int> f0_ranks;
  std::vector<double> f0_cores;
  tnfem_solve_opts opts{};
  std::chrono::steady_clock::time_point t_submit, t_done;
  int state = 0;  // 0 queued, 1 running, 2 done
  int batch = 1;  // size of the lockstep batch it ran in
  int rc = TNFEM_OK;
  std::string error;
  HostTT result;
  tnfem_solve_stats stats{};
  size_t bytes = 0;
};

class Server {
 public:
  Server(int device, int slots, size_t budget) : device_(device), budget_(budget) {
    for (int i = 0; i < slots; ++i) workers_.emplace_back([this] { worker(); });
  }

  ~Server() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_work_.notify_all();
    cv_budget_.notify_all();
    for (auto& t : workers_) t.join();
  }

  long long submit(const tnfem_problem_desc& d, const tnfem_solve_opts& o) {
    auto r = std::make_unique<Request>();
    r->desc = d;
    if (d.layer_E && d.n_layer_E > 0) {
      r->layer.assign(d.layer_E, d.layer_E + d.n_layer_E);
      r->desc.layer_E = r->layer.data();
    }
    if (d.elem_weight && d.n_elem_weight > 0) {
      r->ew.assign(d.elem_weight, d.elem_weight + d.n_elem_weight);
      r->desc.elem_weight = r->ew.data();
    }
    if (d.f0_cores) {
      const size_t nd = f0_doubles(d);  // validates the ranks before they size the copy
      r->f0_ranks.assign(d.f0_ranks, d.f0_ranks + d.level + 2);
      r->f0_cores.assign(d.f0_cores, d.f0_cores + nd);
      r->desc.f0_ranks = r->f0_ranks.data();
      r->desc.f0_cores = r->f0_cores.data();
    }
    r->opts = o;
    r->t_submit = std::chrono::steady_clock::now();
    std::lock_guard<std::mutex> lk(mu_);
    r->id = ++next_id_;
    const long long id = r->id;
    queue_.push_back(r.get());
    all_[id] = std::move(r);
    cv_work_.notify_one();
    return id;
  }

  // Returns nullptr if unknown; blocks until done when wait is set.
  std::unique_ptr<Request> take(long long id, bool wait, bool* busy) {
    std::unique_lock<std::mutex> lk(mu_);
    *busy = false;
    auto it = all_.find(id);
    if (it == all_.end()) return nullptr;
    if (it->second->state != 2) {
      if (!wait) {
        *busy = true;
        return nullptr;
      }
      cv_done_.wait(lk, [&] { return it->second->state == 2; });
    }
    std::unique_ptr<Request> r = std::move(it->second);
    all_.erase(it);
    return r;
  }

  void info(tnfem_server_state* out) {
    std::lock_guard<std::mutex> lk(mu_);
    out->queued = (int)queue_.size();
    out->running = running_;
    out->peak_running = peak_running_;
    out->completed = completed_;
    out->bytes_in_use = in_use_;
    out->peak_bytes = peak_bytes_;
    out->budget_bytes = budget_;
    out->peak_batch = peak_batch_;
    out->batched_requests = batched_;
  }

 private:
  void worker() {
    Context ctx;
    ctx.device = device_;
    if (hipSetDevice(device_) != hipSuccess ||
        hipStreamCreateWithFlags(&ctx.stream, hipStreamNonBlocking) != hipSuccess) {
      return;
    }
    ctx.own_stream = true;
    for (;;) {
      std::vector<Request*> group;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_work_.wait(lk, [&] { return stop_ || !queue_.empty(); });
        if (stop_) break;
        Request* r = queue_.front();
        queue_.pop_front();
        group.push_back(r);
        if (batchable(r))
          for (auto it = queue_.begin(); it != queue_.end() && (int)group.size() < max_batch_;) {
            if (same_bucket(r, *it)) {
              group.push_back(*it);
              it = queue_.erase(it);
            } else {
              ++it;
            }
          }
        for (Request* q : group) q->state = 1;
      }
      if (group.size() == 1) run(ctx, group[0]);
      else run_group(ctx, group);
      {
        std::lock_guard<std::mutex> lk(mu_);
        for (Request* q : group) {
          q->state = 2;
          if (q->batch == 1) q->t_done = std::chrono::steady_clock::now();
          ++completed_;
        }
      }
      cv_done_.notify_all();
    }
    (void)hipStreamSynchronize(ctx.stream);
    if (ctx.scratch) (void)hipFree(ctx.scratch);
    if (ctx.splitk) (void)hipFree(ctx.splitk);
    (void)hipStreamDestroy(ctx.stream);
  }

  // Device bytes of a request: its operator plans and load cores plus the workspace of
  // its rank cap, computed from the host assembly before anything is allocated.
  static size_t request_bytes(const Problem& P, const Request* r) {
    return P.device_bytes + P.workspace_bytes(r->opts.rank_cap, std::max(r->opts.rho, 1));
  }

  void run(Context& ctx, Request* r) {
    std::unique_ptr<Problem> P;
    size_t bytes = 0;
    bool admitted = false;
    try {
      P = make_problem_host(r->desc);
      bytes = request_bytes(*P, r);
      if (bytes > budget_) fail(TNFEM_EBUDGET, "request needs %zu device bytes, budget is %zu", bytes, budget_);
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_budget_.wait(lk, [&] { return stop_ || in_use_ + bytes <= budget_; });
        if (stop_) fail(TNFEM_EBUSY, "server stopped");
        in_use_ += bytes;
        peak_bytes_ = std::max(peak_bytes_, in_use_);
        ++running_;
        peak_running_ = std::max(peak_running_, running_);
        admitted = true;
      }
      r->bytes = bytes;
      upload_problem(&ctx, *P);  // device memory only after admission
      r->rc = run_solve(*P, r->opts, r->result, r->stats);
    } catch (const Error& e) {
      r->rc = e.code;
      r->error = e.what();
    } catch (const std::exception& e) {
      r->rc = TNFEM_EINVAL;
      r->error = e.what();
    }
    P.reset();  // frees the request's device memory before releasing its budget
    if (admitted) {
      std::lock_guard<std::mutex> lk(mu_);
      in_use_ -= bytes;
      --running_;
    }
    cv_budget_.notify_all();
  }

  static bool batchable(const Request* r) {
    return r->opts.ir_max == 0 && r->opts.profile == 0 && r->layer.empty();
  }

  static bool same_bucket(const Request* a, const Request* b) {
    return batchable(b) && a->desc.dim == b->desc.dim && a->desc.level == b->desc.level &&
           std::memcmp(&a->opts, &b->opts, sizeof(tnfem_solve_opts)) == 0;
  }

  // Admits the group's device bytes as one unit (waiting for room in the budget).
  bool admit(size_t bytes) {
    std::unique_lock<std::mutex> lk(mu_);
    cv_budget_.wait(lk, [&] { return stop_ || in_use_ + bytes <= budget_; });
    if (stop_) return false;
    in_use_ += bytes;
    peak_bytes_ = std::max(peak_bytes_, in_use_);
    return true;
  }

  // Runs a bucket as one lockstep batch.  On return `group` holds exactly the
  // requests this worker finished (ran or failed); requests sent back to the queue
  // are removed from it inside the same locked section that requeues them, so a
  // worker that picks them up owns them alone.
  void run_group(Context& ctx, std::vector<Request*>& group) {
    std::vector<std::unique_ptr<Problem>> probs;
    std::vector<Request*> members, mine;
    size_t bytes = 0;
    for (Request* r : group) {
      try {
        auto P = make_problem_host(r->desc);
        const size_t b = request_bytes(*P, r);
        if (b > budget_) fail(TNFEM_EBUDGET, "request needs %zu device bytes, budget is %zu", b, budget_);
        if (bytes + b > budget_) {  // the rest waits for another slot
          std::lock_guard<std::mutex> lk(mu_);
          r->state = 0;
          queue_.push_front(r);
          cv_work_.notify_one();
          continue;  // not in `mine`: another worker may own it from here on
        }
        bytes += b;
        r->bytes = b;
        probs.push_back(std::move(P));
        members.push_back(r);
        mine.push_back(r);
      } catch (const Error& e) {
        r->rc = e.code;
        r->error = e.what();
        r->t_done = std::chrono::steady_clock::now();
        mine.push_back(r);
      }
    }
    group.swap(mine);
    if (members.empty()) return;
    if (!admit(bytes)) {
      for (Request* r : members) {
        r->rc = TNFEM_EBUSY;
        r->error = "server stopped";
      }
      return;
    }
    {
      std::lock_guard<std::mutex> lk(mu_);
      running_ += (int)members.size();
      peak_running_ = std::max(peak_running_, running_);
      peak_batch_ = std::max(peak_batch_, (int)members.size());
      if (members.size() > 1) batched_ += (long long)members.size();
    }
    const auto t0 = std::chrono::steady_clock::now();
    try {
      std::vector<Problem*> ps;
      for (auto& P : probs) {
        upload_problem(&ctx, *P);  // device memory only after admission
        ps.push_back(P.get());
      }
      std::vector<HostTT> outs;
      std::vector<tnfem_solve_stats> st;
      std::vector<int> rcs;
      run_solve_batch(ps, members[0]->opts, outs, st, rcs);
      for (size_t i = 0; i < members.size(); ++i) {
        Request* r = members[i];
        r->rc = rcs[i];
        r->stats = st[i];
        r->result = std::move(outs[i]);
        r->batch = (int)members.size();
        r->t_done = t0 + std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                             std::chrono::duration<double>(st[i].seconds));
      }
    } catch (const Error& e) {
      for (Request* r : members) {
        r->rc = e.code;
        r->error = e.what();
      }
    } catch (const std::exception& e) {
      for (Request* r : members) {
        r->rc = TNFEM_EINVAL;
        r->error = e.what();
      }
    }
    probs.clear();  // frees the group's device memory before releasing its budget
    {
      std::lock_guard<std::mutex> lk(mu_);
      in_use_ -= bytes;
      running_ -= (int)members.size();
    }
    cv_budget_.notify_all();
  }

 public:
  void set_max_batch(int b) {
    std::lock_guard<std::mutex> lk(mu_);
    max_batch_ = b;
  }

 private:
  int device_;
  size_t budget_;
  int max_batch_ = 8;
  int peak_batch_ = 1;
  long long batched_ = 0;
  std::mutex mu_;
  std::condition_variable cv_work_, cv_done_, cv_budget_;
  std::deque<Request*> queue_;
  std::map<long long, std::unique_ptr<Request>> all_;
  std::vector<std::thread> workers_;
  long long next_id_ = 0;
  bool stop_ = false;
  size_t in_use_ = 0, peak_bytes_ = 0;
  int running_ = 0, peak_running_ = 0;
  long long completed_ = 0;
};

}  // namespace tnfem

struct tnfem_server {
  std::unique_ptr<tnfem::Server> s;
};

template <class F>
static int guarded_s(F&& f) {
  try {
    return f();
  } catch (const tnfem::Error& e) {
    tnfem::set_last_error(e.what());
    return e.code;
  } catch (const std::exception& e) {
    tnfem::set_last_error(e.what());
    return TNFEM_EINVAL;
  }
}

extern "C" {

int tnfem_server_create(int device, int slots, size_t hbm_budget_bytes, tnfem_server** out) {
  return guarded_s([&]() -> int {
    if (!out) tnfem::fail(TNFEM_EINVAL, "out is NULL");
    if (slots < 1 || slots > 64) tnfem::fail(TNFEM_EINVAL, "slots must be in [1, 64]");
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) tnfem::fail(TNFEM_EDEVICE, "no HIP device");
    if (device < 0 || device >= count) tnfem::fail(TNFEM_EINVAL, "device out of range");
    size_t budget = hbm_budget_bytes;
    if (budget == 0) {
      size_t free_b = 0, total_b = 0;
      tnfem::hip_check(hipSetDevice(device), "hipSetDevice");
      tnfem::hip_check(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
      budget = (size_t)(0.8 * (double)free_b);
    }
    auto s = std::make_unique<tnfem_server>();
    s->s = std::make_unique<tnfem::Server>(device, slots, budget);
    *out = s.release();
    return TNFEM_OK;
  });
}

int tnfem_server_submit(tnfem_server* s, const tnfem_problem_desc* desc, const tnfem_solve_opts* opts,
                        long long* ticket) {
  return guarded_s([&]() -> int {
    if (!s || !desc || !ticket) tnfem::fail(TNFEM_EINVAL, "NULL argument");
    tnfem_solve_opts o;
    if (opts) o = *opts;
    else tnfem_default_opts(&o);
    *ticket = s->s->submit(*desc, o);
    return TNFEM_OK;
  });
}

int tnfem_server_poll(tnfem_server* s, long long ticket, int wait, tnfem_tt** u_out, tnfem_solve_stats* stats,
                      double* latency_s) {
  return guarded_s([&]() -> int {
    if (!s) tnfem::fail(TNFEM_EINVAL, "NULL server");
    bool busy = false;
    auto r = s->s->take(ticket, wait != 0, &busy);
    if (busy) return TNFEM_EBUSY;
    if (!r) tnfem::fail(TNFEM_EINVAL, "unknown ticket %lld", ticket);
    if (stats) *stats = r->stats;
    if (latency_s) *latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
    if (u_out) *u_out = nullptr;
    if (r->rc == TNFEM_OK || r->rc == TNFEM_ENOTCONV) {
      if (u_out) {
        auto t = new tnfem_tt;
        t->t = std::move(r->result);
        *u_out = t;
      }
    } else {
      tnfem::set_last_error(r->error.c_str());
    }
    return r->rc;
  });
}

int tnfem_server_info(tnfem_server* s, tnfem_server_state* info) {
  return guarded_s([&]() -> int {
    if (!s || !info) tnfem::fail(TNFEM_EINVAL, "NULL argument");
    s->s->info(info);
    return TNFEM_OK;
  });
}

int tnfem_server_set_max_batch(tnfem_server* s, int max_batch) {
  return guarded_s([&]() -> int {
    if (!s) tnfem::fail(TNFEM_EINVAL, "NULL server");
    if (max_batch < 1 || max_batch > tnfem::FB_MAX) tnfem::fail(TNFEM_EINVAL, "max_batch must be in [1, 16]");
    s->s->set_max_batch(max_batch);
    return TNFEM_OK;
  });
}

int tnfem_server_destroy(tnfem_server* s) {
  delete s;
  return TNFEM_OK;
}

}  // extern "C"
