/*
 * C ABI of the MI355X lattice Green's function solver.
 *
 * Problem (Dorschner, Yu, Mengaldo & Colonius, "A fast multi-resolution lattice Green's function
 * method for elliptic difference equations", Sec. 2, discrete Poisson equation and
 * eq. discretConv): L u = f on the unbounded cell-centred lattice, L the 7-point Laplacian
 * (sum of the 6 neighbours - 6 u), supp f a union of Cartesian blocks.  On one uniform level the
 * result is u(n) = sum_m G(n - m) f(m) with the lattice Green's function G, evaluated by the fast
 * lattice Green's function method (Sec. 2.1, Algorithm 1: octree of blocks, Lagrange
 * anterpolation/interpolation, zero-padded block FFT convolutions against LGF spectra).  With
 * refinement levels (Sec. 3, Algorithm 2) each level l has spacing h_l = 2^-l, operator
 * L^l = h_l^-2 (7-point) and kernel h_l^2 G; sources are coarsened onto non-leaf blocks, each
 * level is solved in order with the source correction, and coarse fields are interpolated to
 * the next level.
 *
 * Conventions
 *  - blocks[i] = (bx, by, bz) in units of N_b cells of level levels[i]; cell (x, y, z) of block i
 *    is the level lattice point b N_b + (x, y, z).  A level-(l+1) block's parent is floor(b / 2)
 *    at level l.  Every level-l block with children must have all 8 of them.
 *  - Field arrays f and u are device pointers to [n][N_b][N_b][N_b] doubles, x fastest, in the
 *    order of `blocks`.  f on non-leaf blocks is ignored (recomputed by coarsening);
 *    u on a non-leaf block receives that level's total field.
 *  - Ownership: the caller owns f and u (device memory, e.g. torch tensors).  A plan owns its
 *    layout tables and constants (work-item images, weights); the LGF table and kernel spectra
 *    are process-wide and shared.  The buffers of a solve (source and target spectra, level
 *    fields) form a workspace that is not part of the plan: lgf_solve takes one per stream
 *    (allocated on the first solve on that stream, under the plan's hbm_budget, and kept until
 *    lgf_plan_destroy), the server takes one per admitted request from its own memory.  So
 *    solves of one plan may run concurrently on different streams.
 *  - Errors are returned as lgf_status; nothing throws across the ABI.  HIP launch errors give
 *    LGF_EHIP; asynchronous faults surface at the caller's next synchronisation.
 *  - Solves are asynchronous on the given stream; solves of one plan on one stream run in
 *    stream order.
 */
#ifndef LGF_H_
#define LGF_H_

#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lgf_plan_s* lgf_plan_t;
typedef struct lgf_server_s* lgf_server_t;
typedef void* lgf_stream_t;   /* a hipStream_t; NULL = the default stream */

typedef enum {
  LGF_OK = 0,
  LGF_EINVAL = -1,    /* bad argument (null pointer, size, option) */
  LGF_ELAYOUT = -2,   /* invalid block layout (duplicate, orphan, incomplete children, N_b) */
  LGF_ENOMEM = -3,    /* device allocation failed or HBM budget exceeded */
  LGF_EHIP = -4,      /* HIP runtime or launch error */
  LGF_EBUSY = -5      /* server: request not admitted yet / still running */
} lgf_status;

typedef enum {
  LGF_FP64_PLAIN = 0,   /* FFTs, spectral MAC and operators in FP64 */
  LGF_FP32_REFINE = 1   /* the base octree level of every refinement level (block or super-block
                           FFTs and their MAC, about 95 % of the work) in FP32, the coarse octree
                           levels (far field) in FP64, level fields J w and w in FP64; then
                           dc_iters defect-correction iterations: FP64 residual r = f - L u, an
                           all-FP32 re-solve of r and the FP64 update u += e */
} lgf_precision;

/* How the base octree level of every refinement level is convolved.  Both give the same result
 * up to rounding: every base-level interaction of a block (its near list N(B) and influence list
 * I(B), Sec. 2.1) has its source among the children of the 27 neighbours of the block's parent.
 *   LGF_BASE_SUPER: one zero-padded convolution per parent super-block (2 N_b cells per side,
 *                   FFT size 4 N_b) against the 27 neighbouring super-blocks (default);
 *   LGF_BASE_BLOCK: one zero-padded convolution per block (FFT size 2 N_b) against the up to 216
 *                   blocks of its lists, as the paper describes. */
typedef enum { LGF_BASE_SUPER = 0, LGF_BASE_BLOCK = 1 } lgf_base_level;

typedef struct {
  int32_t precision;     /* lgf_precision */
  int32_t dc_iters;      /* defect-correction iterations for LGF_FP32_REFINE (0..8) */
  int32_t autotune;      /* 1: time the launch shapes of the far-field MAC steps at plan time */
  int32_t base_level;    /* lgf_base_level */
  uint64_t hbm_budget;   /* bytes the plan may hold: its constants plus the workspaces lgf_solve and
                            lgf_solve_batch allocate (one per stream and occurrence); lgf_plan
                            fails with LGF_ENOMEM if constants and one workspace exceed it, a solve
                            that needs one more workspace than fits returns LGF_ENOMEM; 0 = no
                            limit */
} lgf_options;

typedef struct {
  int64_t blocks;             /* blocks in the layout */
  int64_t unknowns;           /* blocks * N_b^3 */
  int32_t refinement_levels;
  int32_t max_octree_levels;
  int64_t interactions;       /* (target, source) block pairs over all FMM levels and channels */
  int64_t fft_forward;        /* forward block FFTs per solve pass */
  int64_t fft_inverse;        /* inverse block FFTs per solve pass */
  int64_t mac_rows;
  int64_t workspace_bytes;    /* device bytes of one solve's workspace (with the item images) */
  int64_t spectra;            /* distinct kernel spectra referenced */
  int64_t super_forward;      /* forward super-block FFTs per solve pass (LGF_BASE_SUPER) */
  int64_t super_inverse;      /* inverse super-block FFTs per solve pass */
  int64_t near_rows;          /* rows of 8 target super-blocks in the base-level MAC */
  int64_t near_pairs;         /* (target, source) super-block pairs in the base-level MAC */
  int64_t mac_lds_tiles;      /* coarse-level MAC tiles that stage their spectra in LDS */
  int64_t mac_lds_inner;      /* of those, tiles whose sources all lie within their rows' x
                                 extent (their products with the window's outer, all-zero
                                 entries are skipped) */
} lgf_plan_info;

/* Builds the FP64 LGF table on the current device (Sec. 2: quadrature of eq. GL_B for
 * |n| <= 100).  Called implicitly by lgf_plan; idempotent. */
lgf_status lgf_init(void);

/* Plans a solve for the block layout.  N_b in {8, 16}; interp_order = n_I Lagrange nodes of the
 * FMM interpolation (Sec. 2.1, n_I <= 10 in the paper), 2 <= n_I <= N_b.  opt may be NULL
 * (FP64 plain).  Copies what it needs from the host arrays; builds kernel spectra on first use. */
lgf_status lgf_plan(const int32_t* blocks, const int32_t* levels, int64_t n, int32_t N_b,
                    int32_t interp_order, const lgf_options* opt, lgf_plan_t* out);

/* u = solution for source f (device pointers, layout above); asynchronous on stream. */
lgf_status lgf_solve(lgf_plan_t p, const double* f, double* u, lgf_stream_t stream);

/* lgf_solve for callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  The solve's workspace is a static device array
 * of LGF_SCRATCH_BYTES in the library, one per GPU, held from the first use on that GPU (or
 * lgf_init) until the process ends, instead of a workspace of the plan's.  Every call places the
 * plan's work items in the array and clears the ranges that must start at zero, on stream, before
 * the solve; it calls no hipMalloc, hipFree or other allocating routine, captures no graph and
 * runs on stream alone.  Results equal lgf_solve's.  The caller passes f and u as for lgf_solve.
 * All calls on one GPU share the array, which keeps the last call's contents: calls that overlap
 * in time on one GPU (other streams, other threads) race and must be serialised by the caller;
 * calls on one stream are ordered by the stream.  LGF_ENOMEM if the plan's workspace
 * (lgf_plan_info.workspace_bytes) exceeds LGF_SCRATCH_BYTES, LGF_EINVAL for a null argument. */
#define LGF_SCRATCH_BYTES ((int64_t)64 << 20)
lgf_status lgf_solve_noalloc(lgf_plan_t p, const double* f, double* u, lgf_stream_t stream);

/* Forward operators on the layout's per-level lattice (Sec. 3: the source correction makes the
 * 7-point operator of each level consistent with the computed inverse, and applications need at
 * least the gradient of the solution), with h = 2^-level base cells.  A neighbour cell across a
 * block face is the same-level block's value; at a level boundary (a level l >= 1 block with no
 * same-level block across the face) it is the ghost value of the block's parent field in u, the
 * parent's quadratic extended one child cell outward (the ghost of the source correction).
 * Evaluated on every leaf cell of levels >= 1 and on the level-0 leaf cells whose neighbours lie
 * in level-0 blocks; every other cell (non-leaf blocks, the coarsest level's outer boundary) is
 * set to 0:
 *   LGF_OP_LAPLACIAN  u [n][N_b^3]     -> out [n][N_b^3]     h^-2 (6 neighbours - 6 centre)
 *   LGF_OP_GRADIENT   u [n][N_b^3]     -> out [3][n][N_b^3]  (u(x + e_a) - u(x - e_a)) / 2h
 *   LGF_OP_CURL       u [3][n][N_b^3]  -> out [3][n][N_b^3]  curl by the same central differences
 * u and out are FP64 device arrays in the block layout of lgf_solve (component-major), owned by
 * the caller and not overlapping; asynchronous on stream.  LGF_EINVAL for a null argument or an
 * unknown op. */
typedef enum { LGF_OP_LAPLACIAN = 0, LGF_OP_GRADIENT = 1, LGF_OP_CURL = 2 } lgf_op;
lgf_status lgf_apply(lgf_plan_t p, int32_t op, const double* u, double* out, lgf_stream_t stream);

/* n independent solves advanced together: every phase of all plans runs in shared launches.
 * A plan may appear several times (e.g. the components of a vector field on one layout): its
 * k-th occurrence runs on the plan's k-th workspace of that stream.  Results equal n separate
 * lgf_solve calls. */
lgf_status lgf_solve_batch(const lgf_plan_t* p, const double* const* f, double* const* u, int32_t n,
                           lgf_stream_t stream);

lgf_status lgf_plan_get_info(lgf_plan_t p, lgf_plan_info* out);

/* Builds the plan on the host only (no device memory, no GPU needed) and checks that every
 * kernel work item stays inside the plan's buffers; fills *info (may be NULL) with the counts
 * lgf_plan_get_info would report.  Returns LGF_OK, a validation code, or LGF_EINVAL if an
 * internal consistency check fails (with a message on stderr). */
lgf_status lgf_plan_check(const int32_t* blocks, const int32_t* levels, int64_t n, int32_t N_b,
                          int32_t interp_order, const lgf_options* opt, lgf_plan_info* info);
lgf_status lgf_plan_destroy(lgf_plan_t p);
const char* lgf_status_string(lgf_status s);

/* Diagnostics used by the tests.
 * lgf_green_eval: out[i] = G(n[i]) with the paper's policy (table / A_G^3 / A_G^2); n is a device
 *   array [m][3] of int32, out a device array [m] of doubles.
 * lgf_green_table: copies the dense table cube [101][101][101] (entries for sorted
 *   a >= b >= c with a^2+b^2+c^2 <= 100^2 are valid) to the device array out.
 * lgf_kernel_spectrum: FP64 half spectrum [2N_b][2N_b][N_b+1] (kx fastest) of the zero-padded
 *   kernel block G(s (d N_b + r)), |d| <= 3, s a power of two, to the device array out (complex
 *   as interleaved doubles).  s = 0 selects the base-level super-block kernels instead: block
 *   side B = 2 N_b, G(d B + r) for |d| <= 1, half spectrum [2B][2B][B+1]. */
lgf_status lgf_green_eval(const int32_t* n, int64_t m, double* out, lgf_stream_t stream);
/* lgf_plan_set_mac_shape: forces the launch shape of the tile spectral MAC steps of p (coarse
 *   octree levels; also the base level with LGF_BASE_BLOCK) whose element type has it: shape 1
 *   one target row per wavefront, 2 two rows, 4 the tile's four rows (FP32 steps), 6 source rows
 *   split over 6 wavefronts (FP64 steps), 8 the tile's rows on 4 wavefronts sharing each source
 *   row through LDS, 16 the LDS form (a workgroup stages a chunk of 16 frequencies of the 172
 *   kernel spectra and of the step's source spectra once, then up to 4 tiles work from LDS;
 *   only coarse steps of rows of 4 whose source slots lie within 64 of each other have it, the
 *   planner's choice there); 0 restores the planner's and autotuner's choice.  So that every
 *   shape can be checked; results agree up to rounding order.  LGF_EINVAL for another value. */
lgf_status lgf_plan_set_mac_shape(lgf_plan_t p, int32_t shape);
/* lgf_plan_set_near_shape: the same for the base-level super-block MAC steps: shape 2, 4 or 8
 *   rows of that many target super-blocks per wavefront, 20 or 22 tiles of 2 x 2 or 2 x 4 rows of 4
 *   (FP32 spectra), 21 or 23 the same tiles pipelined over runs of frequency chunks (FP32 and
 *   FP64 spectra; only where every tile of the step has at most 36 or 48 source super-blocks),
 *   42 or 44 the fused form of those tiles (the step also takes the z transforms of the
 *   super-block FFTs: z transform, MAC and inverse z transform per (kx, ky) line in one kernel;
 *   the default wherever the tiles fit); 0 restores the chosen shape.  Shapes other than the
 *   chosen one and its fused / pipelined counterpart exist only in plans built with
 *   lgf_options.autotune = 1; returns LGF_EINVAL, changing nothing, if a step lacks the shape. */
lgf_status lgf_plan_set_near_shape(lgf_plan_t p, int32_t shape);
lgf_status lgf_green_table(double* out, lgf_stream_t stream);
lgf_status lgf_kernel_spectrum(int32_t N_b, int32_t s, int32_t dx, int32_t dy, int32_t dz,
                               double* out, lgf_stream_t stream);

/* Launch timing (diagnostics for benchmarks).  lgf_profile(1) brackets every subsequent
 * kernel launch with HIP events on its stream; lgf_profile_read synchronises on them and returns
 * one entry per (kernel kind, element type, N_b, launch shape) with the launch count, the summed
 * elapsed time and the summed work (spectral MAC: block interactions), then clears the record.
 * mode is the launch shape (the values of lgf_plan_set_mac_shape / lgf_plan_set_near_shape for
 * the MAC steps, 1 for super-block transforms on line-major planes, else 0).
 * Kinds: 0 coarsen, 1 convert, 2 refine, 3 correct, 4 anterpolate, 5 forward FFT, 6 spectral MAC,
 * 7 inverse FFT, 8 interpolate, 9 combine, 10 residual.  precision: 0 FP32, 1 FP64,
 * 2 FP32 child level / FP64 parent level. */
typedef struct {
  int32_t kind;
  int32_t precision;
  int32_t n_b;
  int32_t mode;
  int64_t launches;
  double ms;
  int64_t work;
} lgf_profile_entry;
lgf_status lgf_profile(int32_t enable);
lgf_status lgf_profile_read(lgf_profile_entry* out, int32_t cap, int32_t* n);

/* Serving: continuous batching of solve requests under an HBM budget.
 * lgf_server_create: hbm_budget bounds the device memory the server takes for request workspaces
 *   (reserved in chunks of up to 16 GiB as requests need it and kept until lgf_server_destroy;
 *   0 = no bound).  Requests are admitted in arrival order while their workspace fits; a request
 *   passed over four times stops later ones from overtaking it.  Each admitted request gets its
 *   own workspace slot, so requests of one plan run concurrently.  A launcher thread enqueues
 *   every admitted request as one multi-plan solve (every kernel step of all members in shared
 *   launches) on the server's stream, while earlier batches still run; requests arriving
 *   meanwhile form the next batch.  A completion thread retires batches in order and frees
 *   their slots.  A request whose workspace exceeds the budget fails with LGF_ENOMEM.
 * lgf_server_submit: enqueues (plan, f, u) and returns at once; the caller keeps the plan, f and
 *   u alive until the request completes.
 * lgf_server_submit_layout: the same for a block layout (arguments as lgf_plan; opt->hbm_budget
 *   is ignored): a planner thread takes the plan from the server's cache keyed by the layout and
 *   options, or builds it (kept for later requests, at most 256 plans, least recently used first
 *   out), so latency includes plan building on a miss.
 * lgf_server_poll: completion (1) or not (0); the request's error if it failed.
 * Latency = completion - submission, reported as p50/p99 over completed requests; points_per_s
 * = unknowns completed / (last completion - first submission).
 * lgf_server_info: memory and plan-cache counters: bytes reserved from HIP, in use and at most in
 *   use, slots in use and at most in use, relocations of item images into slots, cached plans,
 *   cache hits and misses, total and largest plan-build time (ms). */
typedef struct {
  int64_t reserved_bytes;
  int64_t in_use_bytes;
  int64_t peak_in_use_bytes;
  int64_t slots;
  int64_t peak_slots;
  int64_t binds;
  int64_t plans_cached;
  int64_t plan_hits;
  int64_t plan_misses;
  double plan_ms_total;
  double plan_ms_max;
} lgf_server_memory;
lgf_status lgf_server_create(uint64_t hbm_budget, lgf_stream_t stream, lgf_server_t* out);
lgf_status lgf_server_submit(lgf_server_t s, lgf_plan_t p, const double* f, double* u, int64_t* req_id);
lgf_status lgf_server_submit_layout(lgf_server_t s, const int32_t* blocks, const int32_t* levels, int64_t n,
                                    int32_t N_b, int32_t interp_order, const lgf_options* opt, const double* f,
                                    double* u, int64_t* req_id);
lgf_status lgf_server_poll(lgf_server_t s, int64_t req_id, int32_t* done);
lgf_status lgf_server_wait_all(lgf_server_t s);
lgf_status lgf_server_stats(lgf_server_t s, double* p50_us, double* p99_us, double* points_per_s,
                            int64_t* completed);
lgf_status lgf_server_info(lgf_server_t s, lgf_server_memory* out);
/* Starts the statistics afresh (latencies, throughput window, peaks and counters of
 * lgf_server_info), keeping the cached plans and the reserved memory: e.g. after a warm-up. */
lgf_status lgf_server_reset_stats(lgf_server_t s);
lgf_status lgf_server_destroy(lgf_server_t s);

/* Refinement-criterion layout builder (Sec. 3, Convergence subsection, eq. ref_crit), one
 * adaptation step on the GPU.  Input: a layout (blocks [n][3], levels [n], as for lgf_plan) and a
 * field on its cells ([n][N_b^3] doubles, e.g. the vorticity or the source), all device arrays.
 * omega of a block is its largest |value|, omega_max of level l the largest over level l; a
 * level-l block is flagged when l < n_levels - 1 and omega > alpha^(n_levels - 1 - l) omega_max
 * (alpha^k by repeated multiplication; alpha = 1/32 in the paper).  The new layout keeps the
 * base level (level-0 blocks in their order) and, level by level, the 8 children of every
 * flagged block, in the new order of the flagged blocks, child offset (cx, cy, cz) with cz
 * fastest; only blocks of the input layout (where the field is known) can be flagged, so a
 * block loses its children when its criterion fails, and each step adds at most one level.
 * Repeating the step from the base layout with the field on each new layout builds the layout
 * of n_levels refinement levels.  Output: out_blocks [cap][3] and out_levels [cap] (device),
 * *n_out (host) the number of blocks of the new layout; the call synchronises stream.
 * LGF_ENOMEM (with *n_out set) if n_out > cap; LGF_ELAYOUT for a duplicate block, a level
 * outside [0, 16) or N_b not in {8, 16}; LGF_EINVAL for other bad arguments.  Temporary device
 * memory is allocated and freed inside the call. */
lgf_status lgf_layout_adapt(const int32_t* blocks, const int32_t* levels, int64_t n, int32_t N_b,
                            const double* field, int32_t n_levels, double alpha, int32_t* out_blocks,
                            int32_t* out_levels, int64_t cap, int64_t* n_out, lgf_stream_t stream);

/* Diagnostics: with enable = 1 every workspace is filled with 0xFF bytes (NaN) each time a
 * plan's items are placed into it, before the ranges that must read as zero are cleared; a
 * solve that read anything it had not written would then return NaN.  Process-wide. */
lgf_status lgf_workspace_poison(int32_t enable);

#ifdef __cplusplus
}
#endif

#endif /* LGF_H_ */
