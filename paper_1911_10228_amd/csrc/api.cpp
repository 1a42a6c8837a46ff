// extern "C" entry points (include/lgf.h) and the continuous-batching server.
#include "../../include/lgf.h"

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <set>
#include <thread>

#include "plan.hpp"

struct lgf_plan_s {
  lgf::Plan* p;
};

namespace {

lgf_status from_hip(hipError_t e) {
  if (e == hipSuccess) return LGF_OK;
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return LGF_ENOMEM;
  return LGF_EHIP;
}

bool validate_layout(const int32_t* blocks, const int32_t* levels, int64_t n) {
  std::set<std::array<int, 4>> seen;
  for (int64_t i = 0; i < n; ++i) {
    const int l = levels ? levels[i] : 0;
    if (l < 0 || l > 20) return false;
    if (!seen.insert({l, blocks[3 * i], blocks[3 * i + 1], blocks[3 * i + 2]}).second) return false;
  }
  auto fl = [](int v) { return v >= 0 ? v / 2 : -((-v + 1) / 2); };
  for (int64_t i = 0; i < n; ++i) {
    const int l = levels ? levels[i] : 0;
    const int x = blocks[3 * i], y = blocks[3 * i + 1], z = blocks[3 * i + 2];
    if (l > 0 && !seen.count({l - 1, fl(x), fl(y), fl(z)})) return false;
    int kids = 0;
    for (int oc = 0; oc < 8; ++oc)
      kids += (int)seen.count({l + 1, 2 * x + (oc & 1), 2 * y + ((oc >> 1) & 1), 2 * z + ((oc >> 2) & 1)});
    if (kids != 0 && kids != 8) return false;
  }
  return true;
}

}  // namespace

extern "C" {

lgf_status lgf_init(void) {
  lgf::DeviceCtx* c = nullptr;
  return from_hip(lgf::device_ctx(&c));
}

lgf_status lgf_plan(const int32_t* blocks, const int32_t* levels, int64_t n, int32_t N_b,
                    int32_t interp_order, const lgf_options* opt, lgf_plan_t* out) {
  if (!blocks || !out || n <= 0) return LGF_EINVAL;
  *out = nullptr;
  if (N_b != 8 && N_b != 16) return LGF_ELAYOUT;
  if (interp_order < 2 || interp_order > N_b) return LGF_ELAYOUT;
  lgf_options o{};
  if (opt) o = *opt;
  if (o.precision != LGF_FP64_PLAIN && o.precision != LGF_FP32_REFINE) return LGF_EINVAL;
  if (o.dc_iters < 0 || o.dc_iters > 8) return LGF_EINVAL;
  if (o.base_level != LGF_BASE_SUPER && o.base_level != LGF_BASE_BLOCK) return LGF_EINVAL;
  if (!validate_layout(blocks, levels, n)) return LGF_ELAYOUT;
  lgf::Plan* p = nullptr;
  std::string err;
  hipError_t e = lgf::plan_build(blocks, levels, n, N_b, interp_order, o.precision == LGF_FP32_REFINE,
                                 o.dc_iters, o.hbm_budget, &p, &err, false, o.autotune != 0,
                                 o.base_level == LGF_BASE_SUPER);
  if (e != hipSuccess) {
    if (!err.empty()) std::fprintf(stderr, "lgf_plan: %s\n", err.c_str());
    return from_hip(e);
  }
  *out = new lgf_plan_s{p};
  return LGF_OK;
}

lgf_status lgf_plan_check(const int32_t* blocks, const int32_t* levels, int64_t n, int32_t N_b,
                          int32_t interp_order, const lgf_options* opt, lgf_plan_info* info) {
  if (!blocks || n <= 0) return LGF_EINVAL;
  if (N_b != 8 && N_b != 16) return LGF_ELAYOUT;
  if (interp_order < 2 || interp_order > N_b) return LGF_ELAYOUT;
  lgf_options o{};
  if (opt) o = *opt;
  if (o.precision != LGF_FP64_PLAIN && o.precision != LGF_FP32_REFINE) return LGF_EINVAL;
  if (o.dc_iters < 0 || o.dc_iters > 8) return LGF_EINVAL;
  if (o.base_level != LGF_BASE_SUPER && o.base_level != LGF_BASE_BLOCK) return LGF_EINVAL;
  if (!validate_layout(blocks, levels, n)) return LGF_ELAYOUT;
  lgf::Plan* p = nullptr;
  std::string err;
  hipError_t e = lgf::plan_build(blocks, levels, n, N_b, interp_order, o.precision == LGF_FP32_REFINE,
                                 o.dc_iters, o.hbm_budget, &p, &err, /*dry=*/true, o.autotune != 0,
                                 o.base_level == LGF_BASE_SUPER);
  if (e != hipSuccess) {
    if (!err.empty()) std::fprintf(stderr, "lgf_plan_check: %s\n", err.c_str());
    return e == hipErrorOutOfMemory ? LGF_ENOMEM : LGF_EINVAL;
  }
  if (info) {
    lgf_plan_s tmp{p};
    lgf_plan_get_info(&tmp, info);
  }
  lgf::plan_free(p);
  return LGF_OK;
}

lgf_status lgf_solve(lgf_plan_t p, const double* f, double* u, lgf_stream_t stream) {
  if (!p || !f || !u) return LGF_EINVAL;
  std::vector<lgf::Member> m{{p->p, f, u}};
  return from_hip(lgf::solve_members_graph(m, (hipStream_t)stream));
}

lgf_status lgf_apply(lgf_plan_t p, int32_t op, const double* u, double* out, lgf_stream_t stream) {
  if (!p || !u || !out || op < LGF_OP_LAPLACIAN || op > LGF_OP_CURL) return LGF_EINVAL;
  return from_hip(lgf::plan_apply(p->p, op, u, out, (hipStream_t)stream));
}

lgf_status lgf_solve_batch(const lgf_plan_t* p, const double* const* f, double* const* u, int32_t n,
                           lgf_stream_t stream) {
  if (!p || !f || !u || n < 0) return LGF_EINVAL;
  std::vector<lgf::Member> m;
  std::set<lgf::Plan*> seen;
  for (int i = 0; i < n; ++i) {
    if (!p[i] || !f[i] || !u[i]) return LGF_EINVAL;
    if (!seen.insert(p[i]->p).second) return LGF_EINVAL;
    m.push_back({p[i]->p, f[i], u[i]});
  }
  return from_hip(lgf::solve_members_graph(m, (hipStream_t)stream));
}

lgf_status lgf_plan_get_info(lgf_plan_t p, lgf_plan_info* out) {
  if (!p || !out) return LGF_EINVAL;
  const lgf::Plan* q = p->p;
  out->blocks = q->nblocks;
  out->unknowns = q->nblocks * q->nb * q->nb * q->nb;
  out->refinement_levels = q->LR;
  out->max_octree_levels = q->Kmax;
  out->interactions = q->interactions;
  out->fft_forward = q->n_fwd;
  out->fft_inverse = q->n_inv;
  out->mac_rows = q->n_rows;
  out->workspace_bytes = q->bytes + (q->corr ? q->corr->bytes : 0);
  out->spectra = q->n_spectra;
  out->super_forward = q->n_sup_fwd;
  out->super_inverse = q->n_sup_inv;
  out->near_rows = q->n_near_rows;
  out->near_pairs = q->near_pairs;
  return LGF_OK;
}

lgf_status lgf_plan_set_mac_shape(lgf_plan_t p, int32_t shape) {
  if (!p) return LGF_EINVAL;
  const hipError_t e = lgf::plan_set_mac_shape(p->p, shape);
  return e == hipErrorInvalidValue ? LGF_EINVAL : from_hip(e);
}

lgf_status lgf_plan_set_near_shape(lgf_plan_t p, int32_t shape) {
  if (!p) return LGF_EINVAL;
  const hipError_t e = lgf::plan_set_near_shape(p->p, shape);
  return e == hipErrorInvalidValue ? LGF_EINVAL : from_hip(e);
}

lgf_status lgf_plan_destroy(lgf_plan_t p) {
  if (!p) return LGF_EINVAL;
  lgf::plan_free(p->p);
  delete p;
  return LGF_OK;
}

const char* lgf_status_string(lgf_status s) {
  switch (s) {
    case LGF_OK: return "ok";
    case LGF_EINVAL: return "invalid argument";
    case LGF_ELAYOUT: return "invalid block layout";
    case LGF_ENOMEM: return "out of device memory or over the HBM budget";
    case LGF_EHIP: return "HIP runtime error";
    case LGF_EBUSY: return "busy";
  }
  return "unknown status";
}

lgf_status lgf_green_eval(const int32_t* n, int64_t m, double* out, lgf_stream_t stream) {
  if (m < 0 || (m > 0 && (!n || !out))) return LGF_EINVAL;
  lgf::DeviceCtx* c = nullptr;
  hipError_t e = lgf::device_ctx(&c);
  if (e != hipSuccess) return from_hip(e);
  return from_hip(lgf::launch_green_eval(n, m, c->cube, out, (hipStream_t)stream));
}

lgf_status lgf_green_table(double* out, lgf_stream_t stream) {
  if (!out) return LGF_EINVAL;
  lgf::DeviceCtx* c = nullptr;
  hipError_t e = lgf::device_ctx(&c);
  if (e != hipSuccess) return from_hip(e);
  const size_t nb = (size_t)(lgf::kTableKmax + 1) * (lgf::kTableKmax + 1) * (lgf::kTableKmax + 1);
  return from_hip(hipMemcpyAsync(out, c->cube, nb * sizeof(double), hipMemcpyDeviceToDevice,
                                 (hipStream_t)stream));
}

lgf_status lgf_kernel_spectrum(int32_t N_b, int32_t s, int32_t dx, int32_t dy, int32_t dz, double* out,
                               lgf_stream_t stream) {
  const int R = s == 0 ? 1 : 3;
  if (!out || (N_b != 8 && N_b != 16) || s < 0 || (s & (s - 1)) || dx < -R || dx > R || dy < -R ||
      dy > R || dz < -R || dz > R)
    return LGF_EINVAL;
  lgf::DeviceCtx* c = nullptr;
  hipError_t e = lgf::device_ctx(&c);
  if (e != hipSuccess) return from_hip(e);
  const lgf::SpecSet* ss = nullptr;
  e = lgf::spectra_for(c, N_b, s == 0 ? -1 : s, &ss);      // s = 0: base-level super-blocks
  if (e != hipSuccess) return from_hip(e);
  const size_t S = (size_t)ss->spec;
  const int W = 2 * R + 1;
  const int idx = ((dz + R) * W + (dy + R)) * W + (dx + R);
  return from_hip(hipMemcpyAsync(out, ss->d64 + idx * S, S * sizeof(lgf::c64), hipMemcpyDeviceToDevice,
                                 (hipStream_t)stream));
}

lgf_status lgf_profile(int32_t enable) {
  lgf::profile_enable(enable != 0);
  return LGF_OK;
}

lgf_status lgf_profile_read(lgf_profile_entry* out, int32_t cap, int32_t* n) {
  if (!n || (cap > 0 && !out)) return LGF_EINVAL;
  std::vector<lgf::ProfileEntry> v;
  hipError_t e = lgf::profile_collect(&v);
  if (e != hipSuccess) return from_hip(e);
  *n = (int32_t)v.size();
  for (int32_t i = 0; i < std::min<int32_t>(cap, (int32_t)v.size()); ++i) {
    out[i].kind = v[i].kind;
    out[i].precision = v[i].ty;
    out[i].n_b = v[i].nb;
    out[i].launches = v[i].launches;
    out[i].ms = v[i].ms;
    out[i].work = v[i].work;
  }
  return LGF_OK;
}

}  // extern "C"

// ============================================================================= server
// Requests are admitted in arrival order while the workspace of the plans in flight fits the
// budget (one request per plan at a time: a plan's workspace serves one solve).  Each launcher
// step solves every admitted request with shared launches (all phases of all admitted plans
// interleaved by refinement level and phase) and records an event; a completion thread stamps
// the finish time of each request when its step's event has fired.  Requests arriving while a
// step runs join the next step.
struct lgf_server_s {
  struct Req {
    int64_t id;
    lgf::Plan* plan;
    const double* f;
    double* u;
    std::chrono::steady_clock::time_point t0;
  };
  struct Batch {
    hipEvent_t ev;
    std::vector<Req> reqs;
    int64_t bytes;
  };
  uint64_t budget;
  hipStream_t stream;
  std::mutex mu;
  std::condition_variable cv, cv_done;
  std::deque<Req> queue;
  std::deque<Batch> inflight;
  std::set<lgf::Plan*> busy;
  int64_t inflight_bytes = 0;
  std::map<int64_t, int> state;            // 0 queued, 1 running, 2 done, -1 failed
  std::vector<double> lat_us;
  int64_t next_id = 1;
  int64_t points_done = 0;
  std::chrono::steady_clock::time_point first_submit, last_done;
  bool have_first = false;
  bool stop = false;
  bool launcher_done = false;
  int64_t completions = 0;
  lgf_status error = LGF_OK;
  std::thread launcher, completer;

  void launch_loop() {
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      cv.wait(lk, [&] { return stop || !queue.empty(); });
      if (stop && queue.empty()) {
        launcher_done = true;
        cv_done.notify_all();
        return;
      }
      Batch b;
      b.bytes = 0;
      std::deque<Req> rest;
      std::set<lgf::Plan*> in_batch;
      while (!queue.empty()) {
        Req r = queue.front();
        queue.pop_front();
        const int64_t need = r.plan->bytes + (r.plan->corr ? r.plan->corr->bytes : 0);
        const bool fits = budget == 0 || (uint64_t)(inflight_bytes + b.bytes + need) <= budget ||
                          (inflight.empty() && b.reqs.empty());
        if (!fits || busy.count(r.plan) || in_batch.count(r.plan) || (int)b.reqs.size() >= lgf::kMaxSets) {
          rest.push_back(r);
          continue;
        }
        in_batch.insert(r.plan);
        b.bytes += need;
        b.reqs.push_back(r);
      }
      queue.swap(rest);
      if (b.reqs.empty()) {
        // everything queued waits for a plan or budget held by a step in flight
        const int64_t seen = completions;
        cv.wait(lk, [&] { return completions != seen; });
        continue;
      }
      for (const Req& r : b.reqs) {
        busy.insert(r.plan);
        state[r.id] = 1;
      }
      inflight_bytes += b.bytes;
      lk.unlock();
      std::vector<lgf::Member> m;
      for (const Req& r : b.reqs) m.push_back({r.plan, r.f, r.u});
      hipError_t e = lgf::solve_members(m, stream);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&b.ev, hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventRecord(b.ev, stream);
      lk.lock();
      if (e != hipSuccess) {
        error = LGF_EHIP;
        for (const Req& r : b.reqs) {
          state[r.id] = -1;
          busy.erase(r.plan);
        }
        inflight_bytes -= b.bytes;
        ++completions;
        cv_done.notify_all();
        continue;
      }
      inflight.push_back(std::move(b));
      cv_done.notify_all();
    }
  }

  void complete_loop() {
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      cv_done.wait(lk, [&] { return !inflight.empty() || launcher_done; });
      if (inflight.empty()) return;
      Batch b = inflight.front();
      lk.unlock();
      hipError_t e = hipEventSynchronize(b.ev);
      const auto t1 = std::chrono::steady_clock::now();
      (void)hipEventDestroy(b.ev);
      lk.lock();
      inflight.pop_front();
      for (const Req& r : b.reqs) {
        state[r.id] = e == hipSuccess ? 2 : -1;
        busy.erase(r.plan);
        lat_us.push_back(std::chrono::duration<double, std::micro>(t1 - r.t0).count());
        points_done += r.plan->nblocks * r.plan->nb * r.plan->nb * r.plan->nb;
      }
      if (e != hipSuccess) error = LGF_EHIP;
      last_done = t1;
      ++completions;
      inflight_bytes -= b.bytes;
      cv.notify_all();
      cv_done.notify_all();
    }
  }
};

extern "C" {

lgf_status lgf_server_create(uint64_t hbm_budget, lgf_stream_t stream, lgf_server_t* out) {
  if (!out) return LGF_EINVAL;
  auto* s = new lgf_server_s();
  s->budget = hbm_budget;
  s->stream = (hipStream_t)stream;
  s->launcher = std::thread([s] { s->launch_loop(); });
  s->completer = std::thread([s] { s->complete_loop(); });
  *out = s;
  return LGF_OK;
}

lgf_status lgf_server_submit(lgf_server_t s, lgf_plan_t p, const double* f, double* u, int64_t* req_id) {
  if (!s || !p || !f || !u || !req_id) return LGF_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  lgf_server_s::Req r{s->next_id++, p->p, f, u, std::chrono::steady_clock::now()};
  if (!s->have_first) {
    s->first_submit = r.t0;
    s->have_first = true;
  }
  s->state[r.id] = 0;
  s->queue.push_back(r);
  *req_id = r.id;
  s->cv.notify_all();
  return LGF_OK;
}

lgf_status lgf_server_poll(lgf_server_t s, int64_t req_id, int32_t* done) {
  if (!s || !done) return LGF_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->state.find(req_id);
  if (it == s->state.end()) return LGF_EINVAL;
  if (it->second < 0) return LGF_EHIP;
  *done = it->second == 2 ? 1 : 0;
  return LGF_OK;
}

lgf_status lgf_server_wait_all(lgf_server_t s) {
  if (!s) return LGF_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->queue.empty() && s->inflight.empty() && s->busy.empty(); });
  return s->error;
}

lgf_status lgf_server_stats(lgf_server_t s, double* p50_us, double* p99_us, double* points_per_s,
                            int64_t* completed) {
  if (!s) return LGF_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  std::vector<double> v = s->lat_us;
  std::sort(v.begin(), v.end());
  auto pct = [&](double q) {
    if (v.empty()) return 0.0;
    const size_t i = std::min(v.size() - 1, (size_t)std::ceil(q * v.size()) - (q > 0 ? 1 : 0));
    return v[i];
  };
  if (p50_us) *p50_us = pct(0.50);
  if (p99_us) *p99_us = pct(0.99);
  if (points_per_s) {
    const double dt = s->have_first && !v.empty()
                          ? std::chrono::duration<double>(s->last_done - s->first_submit).count()
                          : 0.0;
    *points_per_s = dt > 0 ? (double)s->points_done / dt : 0.0;
  }
  if (completed) *completed = (int64_t)v.size();
  return LGF_OK;
}

lgf_status lgf_server_destroy(lgf_server_t s) {
  if (!s) return LGF_EINVAL;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv.notify_all();
    s->cv_done.notify_all();
  }
  s->launcher.join();
  s->completer.join();
  delete s;
  return LGF_OK;
}

}  // extern "C"
