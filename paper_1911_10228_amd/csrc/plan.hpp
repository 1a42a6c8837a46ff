// Host-side plan of a (multi-resolution) FLGF solve: octree per refinement level and channel,
// interaction rows, slots of the device arenas, and the ordered list of kernel steps.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.hpp"

namespace lgf {

// ----------------------------------------------------------------------------- device context
// Kernel spectra of one block size and level scale.  s >= 1: the 343 offsets |d| <= 3 of blocks of
// nb cells at lattice scale s, index (dz+3)*49+(dy+3)*7+(dx+3).  s <= -1: the 27 neighbour
// offsets |d| <= 1 of super-blocks of 2 nb cells at scale -s, index (dz+1)*9+(dy+1)*3+(dx+1).
struct SpecSet {
  int nb = 0, s = 0;
  int count = 0;                       // 343 or 27
  int64_t spec = 0;                    // complex entries per spectrum
  c64* d64 = nullptr;
  c32* d32 = nullptr;
  const c64** kp64 = nullptr;          // device arrays of count pointers
  const c32** kp32 = nullptr;
};

struct DeviceCtx {
  int device = -1;
  double* cube = nullptr;              // LGF table [101][101][101]
  std::map<std::pair<int, int>, SpecSet> spectra;
  std::mutex mu;
  hipStream_t stream = nullptr;        // plan-time work
  int64_t bytes = 0;                   // table + spectra
};

// Returns the context of the current device, building the LGF table on first use.
hipError_t device_ctx(DeviceCtx** out);
hipError_t spectra_for(DeviceCtx* ctx, int nb, int s, const SpecSet** out);

// ----------------------------------------------------------------------------- steps
enum StepKind : int {
  K_COARSEN = 0, K_CONVERT, K_REFINE, K_CORRECT, K_ANTERP, K_FWD, K_MAC, K_INV, K_INTERP,
  K_COMBINE, K_RESIDUAL, K_SUP_FWD, K_NEAR_MAC, K_SUP_INV, K_COUNT
};

struct Step {
  int l, phase, sub;                   // ordering key: refinement level, phase, sub-step
  int kind;
  int ty;                              // element type: 0 FP32, 1 FP64, 2 FP32 child / FP64 parent
  const void* items;                   // device pointer into the plan's item buffer
  int32_t count;
  const double* w;                     // weight table for the kernel (or nullptr)
  int64_t work;                        // MAC: block interactions in the step (for flop counts)
  int mode;                            // MAC launch shape chosen by the autotuner (0: default)
  int chain;                           // 0 before the level's fork, 1 base super-block path,
                                       // 2 far field, 3 after the join
};

// Optional launch timing: when enabled, every launch is bracketed by HIP events on its stream
// and the elapsed times are accumulated per (kind, element type) at profile_collect().
void profile_enable(bool on);
struct ProfileEntry { int kind, ty, nb; int64_t launches; double ms; int64_t work; };
hipError_t profile_collect(std::vector<ProfileEntry>* out);

struct Plan {
  int nb = 0, n_i = 0, LR = 0, Kmax = 0;
  bool fp32 = false;
  bool super_base = true;              // base level as parent super-blocks (false: per block)
  bool dry = false;                    // host-only build: fake addresses, no device calls
  std::vector<std::pair<uintptr_t, size_t>> ranges;   // every device range items may touch
  uintptr_t next_fake = 0;
  std::map<std::pair<int, int>, SpecSet> dry_spectra;   // fake kernel spectra of a dry build
  int dc_iters = 0;
  int64_t nblocks = 0;
  DeviceCtx* ctx = nullptr;

  bool tune = false;                   // build launch-shape alternatives for the autotuner
  bool all_fp32 = false;               // every octree level and spectrum in FP32 (correction plan)
  bool correction = false;             // run as a defect-correction pass (see conv_corr)
  Plan* corr = nullptr;                // FP32 + DC: the plan of the correction re-solve (owned)
  std::vector<int> base_slot;          // per block: its base-level source slot
  std::vector<Step> pass;              // one solve pass: input field -> output field
  // alternatives of a pass step (index into pass) with another launch shape and its own items
  std::vector<std::pair<size_t, Step>> alt;
  std::vector<Step> residual;          // r = f - L u (FP32 refine only)
  std::vector<int> mac_mode0;          // chosen MAC launch shapes, kept when a shape is forced
  std::vector<Step> near0;             // chosen steps (all of pass), kept when a near shape is forced
  // correction plan: the residual writes its base-level leaf sources in FP32, so its pass runs
  // conv_corr (non-leaf blocks only) in place of pass[conv_idx]
  int64_t conv_idx = -1;
  Step conv_corr{};

  // owned device memory
  std::vector<void*> allocs;
  int64_t bytes = 0;
  double* fe = nullptr;                // coarsened source (multi-level)
  void* jw = nullptr;                  // FP64 [n][N3]: interpolated coarse field J w
  void* w = nullptr;                   // FP64 [n][N3]: leaf-only field of non-leaf blocks
  void* src = nullptr;                 // T [nsrc][N3]
  void* fhat = nullptr;                // cpx<T> [nsrc][S]
  void* uhat = nullptr;                // cpx<T> [ntgt][S]
  void* v = nullptr;                   // T [ntgt][N3]
  void* sfhat = nullptr;               // cpx<T> [nsup_src + 1][S2]: super-block source spectra
  void* suhat = nullptr;               // cpx<T> [nsup_tgt][S2]: super-block target spectra
  double* r = nullptr;                 // DC residual [n][N3]
  double* d_w = nullptr;               // Lagrange matrix [2 nb][nb]
  double* d_w3 = nullptr;              // quadratic refinement table [(2 nb + 2)][4]
  void* d_items = nullptr;
  void* d_ops = nullptr;                // OpItem [n]: the forward operators' block table

  // statistics
  int64_t interactions = 0, n_fwd = 0, n_inv = 0, n_rows = 0, n_spectra = 0;
  int64_t n_sup_fwd = 0, n_sup_inv = 0, n_near_rows = 0, near_pairs = 0;
};

hipError_t plan_build(const int32_t* blocks, const int32_t* levels, int64_t n, int nb, int n_i,
                      bool fp32, int dc_iters, uint64_t budget, Plan** out, std::string* err,
                      bool dry = false, bool autotune = false, bool super_base = true);
void plan_free(Plan* p);
// Forces the launch shape of every coarse-level MAC step (0: back to the chosen ones).
hipError_t plan_set_mac_shape(Plan* p, int shape);
// Forces the launch shape of every base-level super-block MAC step (0: back to the chosen ones).
hipError_t plan_set_near_shape(Plan* p, int shape);

struct Member {
  Plan* p;
  const double* in;
  double* out;
  bool accumulate = false;             // the pass adds its result into out (the DC update u += e)
};
// out = op(u) on the plan's layout: 0 Laplacian, 1 gradient, 2 curl (see launch_fwd_op).
hipError_t plan_apply(Plan* p, int op, const double* u, double* out, hipStream_t st);
// Runs the given step lists of several plans with shared launches, in key order.
hipError_t run_steps(const std::vector<Member>& m, bool residual, hipStream_t st);
// Full solve of several plans (pass, then defect-correction iterations), shared launches.
hipError_t solve_members(const std::vector<Member>& m, hipStream_t st);
// Same, replayed from a captured hipGraph when the same (plan, in, out) set was solved before on
// a non-default stream (launch overhead of a solve's ~30-80 kernels paid once).
hipError_t solve_members_graph(const std::vector<Member>& m, hipStream_t st);
void graph_forget(Plan* p);

}  // namespace lgf
