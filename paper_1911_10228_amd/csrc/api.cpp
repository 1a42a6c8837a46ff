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
#include <cmath>
#include <thread>

#include "plan.hpp"

struct lgf_plan_s {
  lgf::Plan* p;
};

static_assert(LGF_SCRATCH_BYTES == lgf::kScratchBytes, "the header states the static workspace size");

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
  hipError_t e = lgf::device_ctx(&c);
  lgf::Binding* b = nullptr;
  if (e == hipSuccess) e = lgf::scratch_binding(&b);     // the static workspace's address
  return from_hip(e);
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
  lgf::Binding* b = nullptr;
  hipError_t e = lgf::plan_binding(p->p, (hipStream_t)stream, 0, &b);
  if (e != hipSuccess) return from_hip(e);
  std::vector<lgf::Member> m{{p->p, f, u, false, b}};
  return from_hip(lgf::solve_members_graph(m, (hipStream_t)stream));
}

lgf_status lgf_solve_noalloc(lgf_plan_t p, const double* f, double* u, lgf_stream_t stream) {
  if (!p || !f || !u) return LGF_EINVAL;
  if (p->p->bind_bytes > lgf::kScratchBytes) return LGF_ENOMEM;
  lgf::Binding* b = nullptr;
  hipError_t e = lgf::scratch_binding(&b);
  // the array keeps the last call's contents: place the plan's items and clear its zero ranges
  // on every call, in stream order before the solve
  if (e == hipSuccess) e = lgf::bind(p->p, b, (hipStream_t)stream, /*force=*/true);
  if (e != hipSuccess) return from_hip(e);
  std::vector<lgf::Member> m{{p->p, f, u, false, b}};
  return from_hip(lgf::solve_members(m, (hipStream_t)stream, /*one_stream=*/true));
}

lgf_status lgf_apply(lgf_plan_t p, int32_t op, const double* u, double* out, lgf_stream_t stream) {
  if (!p || !u || !out || op < LGF_OP_LAPLACIAN || op > LGF_OP_CURL) return LGF_EINVAL;
  return from_hip(lgf::plan_apply(p->p, op, u, out, (hipStream_t)stream));
}

lgf_status lgf_solve_batch(const lgf_plan_t* p, const double* const* f, double* const* u, int32_t n,
                           lgf_stream_t stream) {
  if (!p || !f || !u || n < 0) return LGF_EINVAL;
  std::vector<lgf::Member> m;
  std::map<lgf::Plan*, int> seen;           // occurrence k of a plan takes its k-th binding
  for (int i = 0; i < n; ++i) {
    if (!p[i] || !f[i] || !u[i]) return LGF_EINVAL;
    lgf::Binding* b = nullptr;
    hipError_t e = lgf::plan_binding(p[i]->p, (hipStream_t)stream, seen[p[i]->p]++, &b);
    if (e != hipSuccess) return from_hip(e);
    m.push_back({p[i]->p, f[i], u[i], false, b});
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
  out->workspace_bytes = q->bind_bytes;
  out->spectra = q->n_spectra;
  out->super_forward = q->n_sup_fwd;
  out->super_inverse = q->n_sup_inv;
  out->near_rows = q->n_near_rows;
  out->near_pairs = q->near_pairs;
  out->mac_lds_tiles = q->n_lds_tiles;
  out->mac_lds_inner = q->n_lds_inner;
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

lgf_status lgf_layout_adapt(const int32_t* blocks, const int32_t* levels, int64_t n, int32_t N_b,
                            const double* field, int32_t n_levels, double alpha, int32_t* out_blocks,
                            int32_t* out_levels, int64_t cap, int64_t* n_out, lgf_stream_t stream) {
  if (!blocks || !levels || !field || !n_out || n <= 0 || cap < 0 || (cap > 0 && (!out_blocks || !out_levels)))
    return LGF_EINVAL;
  if (N_b != 8 && N_b != 16) return LGF_ELAYOUT;
  if (n_levels < 1 || n_levels > 16 || !(alpha > 0.0 && alpha < 1.0)) return LGF_EINVAL;
  const hipError_t e = lgf::layout_adapt(blocks, levels, n, N_b, field, n_levels, alpha, out_blocks, out_levels,
                                         cap, n_out, (hipStream_t)stream);
  if (e == hipErrorInvalidValue) return LGF_ELAYOUT;
  return from_hip(e);
}

lgf_status lgf_workspace_poison(int32_t enable) {
  lgf::set_poison(enable != 0);
  return LGF_OK;
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
    out[i].mode = v[i].mode;
    out[i].launches = v[i].launches;
    out[i].ms = v[i].ms;
    out[i].work = v[i].work;
  }
  return LGF_OK;
}

}  // extern "C"

// ============================================================================= server
// Requests carry a plan (caller-owned, or resolved by layout from the server's plan cache by a
// planner thread) and are admitted in arrival order as workspace slots free up: a slot is a
// range of the server's device memory (grown in chunks of up to 16 GiB within the budget, kept
// while the server lives) that the plan's items are relocated into.  Several
// requests of one plan run at once on distinct slots.  Each launcher step solves every admitted
// request with shared launches (all phases of all admitted plans interleaved by refinement
// level and phase) and records an event; a completion thread stamps the finish time of each
// request when its step's event has fired and returns its slot.  Requests arriving while a
// step runs join the next step.
struct lgf_server_s {
  struct Req {
    int64_t id;
    lgf::Plan* plan;                       // null until the planner resolved the layout
    const double* f;
    double* u;
    std::chrono::steady_clock::time_point t0;
    int skipped = 0;                       // launcher steps that passed this request over
    // layout of a request submitted by layout
    std::vector<int32_t> blocks, levels;
    int32_t nb = 0, order = 0;
    lgf_options opt{};
  };
  struct Slot {
    int region;
    int64_t off, len;
    lgf::Binding* b;
  };
  struct Batch {
    hipEvent_t ev;
    std::vector<Req> reqs;
    std::vector<Slot> slots;
  };
  struct Region {
    uint8_t* base;
    int64_t bytes;
    std::map<int64_t, int64_t> free;       // offset -> length, coalesced
    std::map<int64_t, std::pair<const lgf::Plan*, int64_t>> image;   // offset -> (plan, length)
  };
  struct CachedPlan {
    lgf::Plan* plan;
    int64_t users = 0;                     // queued or running requests
    uint64_t last_use = 0;
  };
  static constexpr int64_t kChunk = (int64_t)16 << 30;
  static constexpr size_t kPlanCacheMax = 256;

  uint64_t budget;
  hipStream_t stream;
  int device = 0;
  std::mutex mu;
  std::condition_variable cv, cv_done, cv_plan;
  std::deque<Req> queue, plan_queue;
  std::deque<Batch> inflight;
  std::vector<Region> regions;
  std::map<std::vector<int32_t>, CachedPlan> plans;   // layout key -> plan
  uint64_t use_clock = 0;
  int64_t reserved = 0, in_use = 0, peak_in_use = 0, slots = 0, peak_slots = 0, binds = 0;
  int64_t plan_hits = 0, plan_misses = 0;
  double plan_ms_total = 0.0, plan_ms_max = 0.0;
  int64_t running = 0;                     // requests in launched steps
  int64_t planning = 0;                    // requests the planner holds
  std::map<int64_t, int> state;            // 0 queued, 1 running, 2 done, -1 failed
  std::vector<double> lat_us;
  int64_t next_id = 1;
  int64_t points_done = 0;
  std::chrono::steady_clock::time_point first_submit, last_done;
  bool have_first = false;
  bool stop = false;
  bool planner_done = false, launcher_done = false;
  int64_t completions = 0;
  lgf_status error = LGF_OK;
  std::thread planner, launcher, completer;

  static std::vector<int32_t> layout_key(const Req& r) {
    std::vector<int32_t> k{r.nb, r.order, r.opt.precision, r.opt.dc_iters, r.opt.autotune, r.opt.base_level};
    k.insert(k.end(), r.blocks.begin(), r.blocks.end());
    k.insert(k.end(), r.levels.begin(), r.levels.end());
    return k;
  }

  // first fit over the regions; a new chunk while the budget allows.  Called with mu held.
  bool take(int64_t need, Slot* out) {
    need = (need + 255) / 256 * 256;
    for (int pass = 0; pass < 2; ++pass) {
      for (size_t ri = 0; ri < regions.size(); ++ri) {
        Region& R = regions[ri];
        for (auto it = R.free.begin(); it != R.free.end(); ++it) {
          if (it->second < need) continue;
          const int64_t off = it->first, rest = it->second - need;
          R.free.erase(it);
          if (rest) R.free[off + need] = rest;
          out->region = (int)ri;
          out->off = off;
          out->len = need;
          return true;
        }
      }
      if (pass == 1) break;
      const int64_t left = budget ? (int64_t)budget - reserved : INT64_MAX;
      if (left < need) return false;
      const int64_t sz = std::max(need, std::min(left, kChunk));
      void* base = nullptr;
      if (hipMalloc(&base, (size_t)sz) != hipSuccess) {
        // a smaller chunk if the device cannot give the larger one
        if (sz == need || hipMalloc(&base, (size_t)need) != hipSuccess) return false;
        regions.push_back({(uint8_t*)base, need, {{0, need}}, {}});
        reserved += need;
        continue;
      }
      regions.push_back({(uint8_t*)base, sz, {{0, sz}}, {}});
      reserved += sz;
    }
    return false;
  }

  void give_back(const Slot& sl) {
    Region& R = regions[sl.region];
    int64_t off = sl.off, len = sl.len;
    auto nx = R.free.lower_bound(off);
    if (nx != R.free.end() && nx->first == off + len) {
      len += nx->second;
      nx = R.free.erase(nx);
    }
    if (nx != R.free.begin()) {
      auto pv = std::prev(nx);
      if (pv->first + pv->second == off) {
        off = pv->first;
        len += pv->second;
        R.free.erase(pv);
      }
    }
    R.free[off] = len;
  }

  // the binding of a slot for plan p: the plan's item images stay valid where the same plan
  // used the same range last (a solve writes neither its items nor its zero ranges)
  lgf::Binding* slot_binding(Slot& sl, const lgf::Plan* p) {
    Region& R = regions[sl.region];
    const lgf::Plan* have = nullptr;
    for (auto it = R.image.begin(); it != R.image.end();) {
      const int64_t o = it->first, l = it->second.second;
      if (o < sl.off + sl.len && sl.off < o + l) {
        if (o == sl.off && l == sl.len) have = it->second.first;
        it = R.image.erase(it);
      } else {
        ++it;
      }
    }
    R.image[sl.off] = {p, sl.len};
    return new lgf::Binding{R.base + sl.off, sl.len, have, false};
  }

  void fail(const Req& r, lgf_status why) {
    state[r.id] = -1;
    error = why;
    ++completions;
    cv_done.notify_all();
  }

  void release_plan(lgf::Plan* p) {
    for (auto& kv : plans)
      if (kv.second.plan == p) {
        --kv.second.users;
        break;
      }
  }

  void plan_loop() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      cv_plan.wait(lk, [&] { return stop || !plan_queue.empty(); });
      if (plan_queue.empty()) {
        planner_done = true;
        cv.notify_all();
        return;
      }
      Req r = std::move(plan_queue.front());
      plan_queue.pop_front();
      ++planning;
      const std::vector<int32_t> key = layout_key(r);
      auto it = plans.find(key);
      if (it != plans.end()) {
        ++plan_hits;
      } else {
        lk.unlock();
        const auto t0 = std::chrono::steady_clock::now();
        lgf::Plan* p = nullptr;
        std::string err;
        hipError_t e = lgf::plan_build(r.blocks.data(), r.levels.data(), (int64_t)r.levels.size(), r.nb, r.order,
                                       r.opt.precision == LGF_FP32_REFINE, r.opt.dc_iters, 0, &p, &err, false,
                                       r.opt.autotune != 0, r.opt.base_level == LGF_BASE_SUPER);
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        lk.lock();
        if (e == hipSuccess) e = lgf::plan_trim(p);     // the tuning workspace: slots serve the plan
        if (e != hipSuccess) {
          lgf::plan_free(p);
          --planning;
          fail(r, from_hip(e));
          continue;
        }
        ++plan_misses;
        plan_ms_total += ms;
        plan_ms_max = std::max(plan_ms_max, ms);
        // evict the least recently used plans that no request holds
        while (plans.size() >= kPlanCacheMax) {
          auto victim = plans.end();
          for (auto q = plans.begin(); q != plans.end(); ++q)
            if (q->second.users == 0 && (victim == plans.end() || q->second.last_use < victim->second.last_use))
              victim = q;
          if (victim == plans.end()) break;
          for (Region& R : regions)
            for (auto q = R.image.begin(); q != R.image.end();)
              q = q->second.first == victim->second.plan ? R.image.erase(q) : std::next(q);
          lgf::plan_free(victim->second.plan);
          plans.erase(victim);
        }
        it = plans.emplace(key, CachedPlan{p, 0, 0}).first;
      }
      it->second.users += 1;
      it->second.last_use = ++use_clock;
      r.plan = it->second.plan;
      r.blocks.clear();
      r.levels.clear();
      queue.push_back(std::move(r));
      --planning;
      cv.notify_all();
    }
  }

  void launch_loop() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      cv.wait(lk, [&] { return (stop && planner_done) || !queue.empty(); });
      if (queue.empty()) {
        launcher_done = true;
        cv_done.notify_all();
        return;
      }
      Batch b;
      std::deque<Req> rest;
      bool blocked = false;                // an old request waits: admit nothing past it
      while (!queue.empty()) {
        Req r = std::move(queue.front());
        queue.pop_front();
        const int64_t need = r.plan->bind_bytes;
        if (budget && (uint64_t)need > budget) {          // can never be admitted
          release_plan(r.plan);
          fail(r, LGF_ENOMEM);
          continue;
        }
        Slot sl{};
        if (blocked || (int)b.reqs.size() >= lgf::kMaxSets || !take(need, &sl)) {
          if (!blocked && ++r.skipped >= 4) blocked = true;
          rest.push_back(std::move(r));
          continue;
        }
        sl.b = slot_binding(sl, r.plan);
        b.slots.push_back(sl);
        b.reqs.push_back(std::move(r));
      }
      queue.swap(rest);
      if (b.reqs.empty()) {
        if (queue.empty()) continue;       // every request was rejected: wait for more
        // everything queued waits for slots held by a step in flight
        const int64_t seen = completions;
        if (running == 0) {
          // nothing in flight: every region is free.  Chunks taken for earlier sizes may still
          // be too small for the head request; give them back once and retry, else it cannot fit.
          if (!regions.empty()) {
            (void)hipStreamSynchronize(stream);
            for (Region& R : regions) (void)hipFree(R.base);
            regions.clear();
            reserved = 0;
            continue;
          }
          Req r = std::move(queue.front());
          queue.pop_front();
          release_plan(r.plan);
          fail(r, LGF_ENOMEM);
          continue;
        }
        cv.wait(lk, [&] { return completions != seen; });
        continue;
      }
      for (size_t i = 0; i < b.reqs.size(); ++i) {
        state[b.reqs[i].id] = 1;
        in_use += b.slots[i].len;
        ++slots;
      }
      peak_in_use = std::max(peak_in_use, in_use);
      peak_slots = std::max(peak_slots, slots);
      running += (int64_t)b.reqs.size();
      lk.unlock();
      std::vector<lgf::Member> m;
      hipError_t e = hipSuccess;
      int64_t nbind = 0;
      for (size_t i = 0; i < b.reqs.size() && e == hipSuccess; ++i) {
        nbind += b.slots[i].b->plan != b.reqs[i].plan;
        e = lgf::bind(b.reqs[i].plan, b.slots[i].b, stream);
        m.push_back({b.reqs[i].plan, b.reqs[i].f, b.reqs[i].u, false, b.slots[i].b});
      }
      if (e == hipSuccess) e = lgf::solve_members(m, stream);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&b.ev, hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventRecord(b.ev, stream);
      lk.lock();
      binds += nbind;
      if (e != hipSuccess) {
        for (size_t i = 0; i < b.reqs.size(); ++i) {
          fail(b.reqs[i], LGF_EHIP);
          release_plan(b.reqs[i].plan);
          in_use -= b.slots[i].len;
          --slots;
          give_back(b.slots[i]);
          delete b.slots[i].b;
        }
        running -= (int64_t)b.reqs.size();
        continue;
      }
      inflight.push_back(std::move(b));
      cv_done.notify_all();
    }
  }

  void complete_loop() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      cv_done.wait(lk, [&] { return !inflight.empty() || launcher_done; });
      if (inflight.empty()) return;
      Batch b = std::move(inflight.front());
      inflight.pop_front();
      lk.unlock();
      hipError_t e = hipEventSynchronize(b.ev);
      const auto t1 = std::chrono::steady_clock::now();
      (void)hipEventDestroy(b.ev);
      lk.lock();
      for (size_t i = 0; i < b.reqs.size(); ++i) {
        const Req& r = b.reqs[i];
        state[r.id] = e == hipSuccess ? 2 : -1;
        lat_us.push_back(std::chrono::duration<double, std::micro>(t1 - r.t0).count());
        points_done += r.plan->nblocks * r.plan->nb * r.plan->nb * r.plan->nb;
        release_plan(r.plan);
        in_use -= b.slots[i].len;
        --slots;
        give_back(b.slots[i]);
        delete b.slots[i].b;
      }
      running -= (int64_t)b.reqs.size();
      if (e != hipSuccess) error = LGF_EHIP;
      last_done = t1;
      ++completions;
      cv.notify_all();
      cv_done.notify_all();
    }
  }

  Req new_req(const double* f, double* u) {
    Req r;
    r.id = next_id++;
    r.plan = nullptr;
    r.f = f;
    r.u = u;
    r.t0 = std::chrono::steady_clock::now();
    if (!have_first) {
      first_submit = r.t0;
      have_first = true;
    }
    state[r.id] = 0;
    return r;
  }
};

extern "C" {

lgf_status lgf_server_create(uint64_t hbm_budget, lgf_stream_t stream, lgf_server_t* out) {
  if (!out) return LGF_EINVAL;
  auto* s = new lgf_server_s();
  s->budget = hbm_budget;
  s->stream = (hipStream_t)stream;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return LGF_EHIP;
  }
  s->planner = std::thread([s] { s->plan_loop(); });
  s->launcher = std::thread([s] { s->launch_loop(); });
  s->completer = std::thread([s] { s->complete_loop(); });
  *out = s;
  return LGF_OK;
}

lgf_status lgf_server_submit(lgf_server_t s, lgf_plan_t p, const double* f, double* u, int64_t* req_id) {
  if (!s || !p || !f || !u || !req_id) return LGF_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  lgf_server_s::Req r = s->new_req(f, u);
  r.plan = p->p;
  *req_id = r.id;
  s->queue.push_back(std::move(r));
  s->cv.notify_all();
  return LGF_OK;
}

lgf_status lgf_server_submit_layout(lgf_server_t s, const int32_t* blocks, const int32_t* levels, int64_t n,
                                    int32_t N_b, int32_t interp_order, const lgf_options* opt, const double* f,
                                    double* u, int64_t* req_id) {
  if (!s || !blocks || n <= 0 || !f || !u || !req_id) return LGF_EINVAL;
  if (N_b != 8 && N_b != 16) return LGF_ELAYOUT;
  if (interp_order < 2 || interp_order > N_b) return LGF_ELAYOUT;
  lgf_options o{};
  if (opt) o = *opt;
  if (o.precision != LGF_FP64_PLAIN && o.precision != LGF_FP32_REFINE) return LGF_EINVAL;
  if (o.dc_iters < 0 || o.dc_iters > 8) return LGF_EINVAL;
  if (o.base_level != LGF_BASE_SUPER && o.base_level != LGF_BASE_BLOCK) return LGF_EINVAL;
  if (!validate_layout(blocks, levels, n)) return LGF_ELAYOUT;
  std::lock_guard<std::mutex> lk(s->mu);
  lgf_server_s::Req r = s->new_req(f, u);
  r.blocks.assign(blocks, blocks + 3 * n);
  r.levels.assign((size_t)n, 0);
  if (levels) r.levels.assign(levels, levels + n);
  r.nb = N_b;
  r.order = interp_order;
  r.opt = o;
  r.opt.hbm_budget = 0;
  *req_id = r.id;
  s->plan_queue.push_back(std::move(r));
  s->cv_plan.notify_all();
  return LGF_OK;
}

lgf_status lgf_server_poll(lgf_server_t s, int64_t req_id, int32_t* done) {
  if (!s || !done) return LGF_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->state.find(req_id);
  if (it == s->state.end()) return LGF_EINVAL;
  if (it->second < 0) return s->error == LGF_OK ? LGF_EHIP : s->error;
  *done = it->second == 2 ? 1 : 0;
  return LGF_OK;
}

lgf_status lgf_server_wait_all(lgf_server_t s) {
  if (!s) return LGF_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] {
    return s->plan_queue.empty() && s->planning == 0 && s->queue.empty() && s->inflight.empty() &&
           s->running == 0;
  });
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

lgf_status lgf_server_info(lgf_server_t s, lgf_server_memory* out) {
  if (!s || !out) return LGF_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  out->reserved_bytes = s->reserved;
  out->in_use_bytes = s->in_use;
  out->peak_in_use_bytes = s->peak_in_use;
  out->slots = s->slots;
  out->peak_slots = s->peak_slots;
  out->binds = s->binds;
  out->plans_cached = (int64_t)s->plans.size();
  out->plan_hits = s->plan_hits;
  out->plan_misses = s->plan_misses;
  out->plan_ms_total = s->plan_ms_total;
  out->plan_ms_max = s->plan_ms_max;
  return LGF_OK;
}

lgf_status lgf_server_reset_stats(lgf_server_t s) {
  if (!s) return LGF_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  s->lat_us.clear();
  s->points_done = 0;
  s->have_first = false;
  s->peak_in_use = s->in_use;
  s->peak_slots = s->slots;
  s->binds = 0;
  s->plan_hits = s->plan_misses = 0;
  s->plan_ms_total = s->plan_ms_max = 0.0;
  return LGF_OK;
}

lgf_status lgf_server_destroy(lgf_server_t s) {
  if (!s) return LGF_EINVAL;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv.notify_all();
    s->cv_plan.notify_all();
    s->cv_done.notify_all();
  }
  s->planner.join();
  s->launcher.join();
  s->completer.join();
  (void)hipStreamSynchronize(s->stream);
  for (auto& kv : s->plans) lgf::plan_free(kv.second.plan);
  for (auto& R : s->regions) (void)hipFree(R.base);
  delete s;
  return LGF_OK;
}

}  // extern "C"
