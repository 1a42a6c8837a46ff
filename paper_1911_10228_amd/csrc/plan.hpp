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
  c64* col64 = nullptr;                // super-block sets: kernel columns of the fused near step
  c32* col32 = nullptr;                // [14][line][kz], FP64 and FP32
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
  int64_t items;                       // byte offset of the step's items in the plan's item image
  int32_t count;
  const double* w;                     // weight table for the kernel (or nullptr)
  int64_t work;                        // MAC: block interactions in the step (for flop counts)
  int mode;                            // MAC launch shape chosen by the autotuner (0: default)
  int chain;                           // 0 before the level's fork, 1 base super-block path,
                                       // 2 far field, 3 after the join
  bool lds = false;                    // MAC step whose tiles take the kMacLds form (rows of 4,
                                       // source slots within kMacLdsSrc of each other)
};

// Optional launch timing: when enabled, every launch is bracketed by HIP events on its stream
// and the elapsed times are accumulated per (kind, element type) at profile_collect().
void profile_enable(bool on);
struct ProfileEntry { int kind, ty, nb, mode; int64_t launches; double ms; int64_t work; };
hipError_t profile_collect(std::vector<ProfileEntry>* out);

// ----------------------------------------------------------------------------- workspace
// A solve's buffers (source blocks and spectra, target spectra and fields, the coarsened source,
// J w, w, the residual) form the plan's workspace.  Work items address it at virtual addresses
// kVBase + offset; before a solve the items are copied into a Binding -- a device range holding
// [workspace | item images] -- and every virtual pointer in them is moved by (base - kVBase).
// So a plan holds only its layout tables and constants, and any number of solves of one plan can
// run at once on distinct bindings.  The tag in the top 16 bits cannot occur in a non-pointer
// item field (slot indices, counts, masks, offsets below 2^40, doubles of moderate size), which
// the plan build checks by scanning every item word against the pointer fields it relocates.
constexpr uint64_t kVBase = 0x5A5A000000000000ull;
constexpr int kVTagShift = 48;

struct Plan;
struct Binding {
  uint8_t* base = nullptr;             // device range, 256-byte aligned
  int64_t bytes = 0;                   // capacity
  const Plan* plan = nullptr;          // plan whose items are relocated here (nullptr: none)
  bool owned = false;                  // allocated with hipMalloc by the plan (freed with it)
};

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

  // owned device memory (constants: weight tables, the item template, relocation table, the
  // forward operators' block table)
  std::vector<void*> allocs;
  int64_t bytes = 0;                   // constant bytes
  // workspace (virtual addresses, see Binding); the correction plan's workspace comes first in
  // the same virtual range, so one binding serves both
  int64_t vnext = 0;                   // end of the virtual workspace so far (offset from kVBase)
  int64_t ws_bytes = 0;                // this plan's workspace end (main plan: whole range)
  std::vector<std::pair<int64_t, int64_t>> zero;   // workspace ranges (offset, bytes) read as zero
  std::vector<uint8_t> h_items;        // item image with virtual addresses (host)
  void* d_items = nullptr;             // the same image on the device (relocation source)
  std::vector<uint32_t> relocs;        // 8-byte words of the image holding virtual addresses
  uint32_t* d_relocs = nullptr;
  int64_t items_at = 0;                // offset of this plan's item image in a binding
  int64_t bind_bytes = 0;              // binding size (main plan: workspace + both images)
  uint64_t budget = 0;                 // bytes the plan may hold (constants + own bindings)
  // bindings the plan allocated for lgf_solve / lgf_solve_batch: per (stream, occurrence)
  std::mutex bmu;
  std::map<std::pair<hipStream_t, int>, Binding*> bindings;
  std::vector<Binding*> idle;          // allocated but not tied to a stream (plan-time tuning)
  int64_t bound_bytes = 0;
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
  void* d_ops = nullptr;                // OpItem [n]: the forward operators' block table

  // statistics
  int64_t interactions = 0, n_fwd = 0, n_inv = 0, n_rows = 0, n_spectra = 0;
  int64_t n_sup_fwd = 0, n_sup_inv = 0, n_near_rows = 0, near_pairs = 0;
  int64_t n_lds_tiles = 0, n_lds_inner = 0;   // coarse MAC tiles of the LDS form, inner-window ones
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
  Binding* b = nullptr;                // workspace of the solve (the main plan's binding)
};

// Relocates p's item images (and its correction plan's) into b and clears b's zero ranges,
// asynchronously on st, unless b already holds p's images.  With set_poison(true) the workspace
// is first filled with 0xFF bytes (NaN) on every bind (diagnostics: a solve must read nothing it
// has not written).
hipError_t bind(Plan* p, Binding* b, hipStream_t st, bool force = false);
// The binding of p for occurrence k of the plan in a solve on stream st, allocated (under the
// plan's budget) and bound on first use.
hipError_t plan_binding(Plan* p, hipStream_t st, int k, Binding** out);
void set_poison(bool on);
// The static workspace of the allocation-free solve on the current device (a binding of
// kScratchBytes at that device's copy of the array; set up on first use per device).
constexpr int64_t kScratchBytes = (int64_t)64 << 20;
hipError_t scratch_binding(Binding** out);
// Frees the bindings p allocated (after the device finished with them).
hipError_t plan_trim(Plan* p);
// device address of a workspace buffer (virtual address v of p's workspace) in binding b
inline const void* in_binding(const Binding* b, const void* v) {
  return b->base + ((uint64_t)(uintptr_t)v - kVBase);
}
// out = op(u) on the plan's layout: 0 Laplacian, 1 gradient, 2 curl (see launch_fwd_op).
hipError_t plan_apply(Plan* p, int op, const double* u, double* out, hipStream_t st);
// Runs the given step lists of several plans with shared launches, in key order.
// one_stream: no second stream for the base-level path (and no stream or event creation).
hipError_t run_steps(const std::vector<Member>& m, bool residual, hipStream_t st, bool one_stream = false);
// Full solve of several plans (pass, then defect-correction iterations), shared launches.
hipError_t solve_members(const std::vector<Member>& m, hipStream_t st, bool one_stream = false);
// Same, replayed from a captured hipGraph when the same (plan, in, out) set was solved before on
// a non-default stream (launch overhead of a solve's ~30-80 kernels paid once).
hipError_t solve_members_graph(const std::vector<Member>& m, hipStream_t st);
void graph_forget(Plan* p);

}  // namespace lgf
