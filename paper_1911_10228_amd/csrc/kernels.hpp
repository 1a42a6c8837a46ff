// Device work items and kernel launchers of the LGF library.
#pragma once

#include "common.hpp"
#include "fft.hpp"

namespace lgf {

constexpr int kTableKmax = 100;           // table holds |n_i| <= 100 (n.n <= 100^2)
constexpr int kMacL = 8;                  // target blocks per MAC row (x run, starts even)
constexpr int kMacSlots = kMacL + 6;      // source x slots per (dy, dz) pair
constexpr int kMacHalfRows = 32;          // MAC mode bit: tiles of rows of kMacL / 2 targets
constexpr int kMacLds = 16;               // MAC mode: kernel and source spectra of a frequency chunk in LDS
constexpr int kMacLdsSrc = 64;            // at most this many source slots per step for kMacLds

// ----------------------------------------------------------------------------- Green function
// Paper's policy: table for n.n <= 100^2, A_G^3 up to 600^2, A_G^2 beyond.
__device__ __forceinline__ double green(int nx, int ny, int nz, const double* __restrict__ cube) {
  int a = nx < 0 ? -nx : nx, b = ny < 0 ? -ny : ny, c = nz < 0 ? -nz : nz;
  const long r2 = (long)a * a + (long)b * b + (long)c * c;
  if (r2 <= 10000) {
    if (a < b) { int t = a; a = b; b = t; }
    if (b < c) { int t = b; b = c; c = t; }
    if (a < b) { int t = a; a = b; b = t; }
    return cube[((size_t)a * (kTableKmax + 1) + b) * (kTableKmax + 1) + c];
  }
  const double x2 = double(nx) * nx, y2 = double(ny) * ny, z2 = double(nz) * nz;
  const double rr = x2 + y2 + z2;
  const double r = sqrt(rr);
  const double inv_r = 1.0 / r;
  const double inv_r2 = inv_r * inv_r;
  const double inv_r4 = inv_r2 * inv_r2;
  const double quart = x2 * x2 + y2 * y2 + z2 * z2 - 3.0 * (x2 * y2 + x2 * z2 + y2 * z2);
  double g = -inv_r / (4.0 * kPi) - quart * inv_r4 * inv_r2 * inv_r / (16.0 * kPi);
  if (r2 <= 360000) {
    const double oct = -228.0 * (y2 * z2 * x2 * x2 + y2 * z2 * z2 * x2 + y2 * y2 * z2 * x2) +
                       621.0 * (x2 * x2 * y2 * y2 + z2 * z2 * y2 * y2 + x2 * x2 * z2 * z2) -
                       244.0 * (y2 * x2 * x2 * x2 + z2 * x2 * x2 * x2 + y2 * y2 * y2 * x2 +
                                z2 * z2 * z2 * x2 + y2 * z2 * z2 * z2 + y2 * y2 * y2 * z2) +
                       23.0 * (x2 * x2 * x2 * x2 + y2 * y2 * y2 * y2 + z2 * z2 * z2 * z2);
    const double inv_r13 = inv_r4 * inv_r4 * inv_r4 * inv_r;
    g -= oct * inv_r13 / (128.0 * kPi);
  }
  return g;
}

// ----------------------------------------------------------------------------- work items
template <typename T> struct FftFwdItem {
  const T* src;          // n_b^3 real block [z][y][x]
  cpx<T>* dst;           // half spectrum [kz][ky][kx], kx in [0, n_b]
};
template <typename T> struct FftInvItem {
  const cpx<T>* src;     // half spectrum
  T* dst;                // n_b^3 real block, receives IFFT / P^3
};
// A MAC tile: the 2x2 sibling rows y in {2py, 2py+1}, z in {2pz, 2pz+1} of an x window of W
// blocks (8, or 4 with the kMacHalfRows launch bit) starting at x0 = W wx.  Siblings share their
// parent's neighbours, so all four rows draw from the same 6x6 source rows y' = 2py-2+jy,
// z' = 2pz-2+jz (jy, jz in 0..5).  With W = 4 only the first 4 targets and 10 source slots of a
// row are used (the rest are -1 / the zero spectrum).
template <typename T> struct MacTile {
  int32_t tgt[4][kMacL];               // target slots of row r = ry + 2 rz, x = x0 + i (-1: none)
  int32_t src[36][kMacSlots];          // source slots of source row jz*6+jy, x' = x0 - 3 + s
                                       // (absent sources: the arena's all-zero spectrum)
  uint64_t pair_mask;                  // bit jz*6+jy set if that source row has a source
  int32_t flags;                       // bit0: base level (near field included); bit1: every
                                       // source of the tile lies within its rows' x extent
                                       // (LDS form: x0 .. x0 + 3)
  int32_t row_mask;                    // bit r set if row r has a target
  int32_t src_lo, src_n;               // the step's source slots lie in [src_lo, src_lo + src_n)
                                       // (src_n = 0: more than kMacLdsSrc slots; no LDS form)
  const cpx<T>* fhat;                  // source spectra arena (slot * S)
  cpx<T>* uhat;                        // target spectra arena (slot * S)
  const cpx<T>* const* kptr;           // 343 kernel spectra of the tile's level, (dz+3)*49+(dy+3)*7+dx+3
};
// Base-level super-blocks (the 2x2x2 children of one parent, side B2 = 2 N_b, FFT size P = 2 B2)
template <typename T> struct SuperFwdItem {
  const T* child[8];     // child source blocks, octant cx + 2 cy + 4 cz (nullptr: see child_in)
  int64_t child_in[8];   // where child is null: offset of the child in WorkSet::in (FP64
                         // children only), -1: zero
  cpx<T>* tmp;           // intermediate planes [B2][P][B2+1]
  cpx<T>* dst;           // super-block half spectrum [P][P][B2+1]
};
template <typename T> struct SuperInvItem {
  const cpx<T>* src;     // super-block half spectrum
  cpx<T>* tmp;           // intermediate planes
  T* child[8];           // child field blocks receiving the cropped IFFT / P^3 (nullptr: skip)
};
constexpr int kNearSlots = kMacL + 2;     // source x slots of a near row: x0 - 1 .. x0 + W
// A near row: up to W (4 or 8) super-block targets along x starting at x0 = W wx; each interacts
// with the 27 super-blocks at offsets |D|_inf <= 1 through the exact base-lattice kernel.  The
// non-empty source rows (dy, dz) are listed first, padded with all-zero rows to a multiple of 3.
template <typename T> struct NearRow {
  int32_t tgt[kMacL];                  // target super slots (-1: none), first W used
  int32_t src[9][kNearSlots];          // source super slots of listed row i at x0 - 1 + q, q < W + 2
                                       // (the zero slot where absent)
  uint64_t pj_code;                    // listed row i is source row (dz+1)*3+(dy+1) =
                                       // bits [4 i, 4 i + 4) (one scalar word: no per-row loads)
  int32_t ngroups;                     // listed rows / 3
  int32_t pad;
  const cpx<T>* fhat;                  // super source spectra arena (slot * S)
  cpx<T>* uhat;                        // super target spectra arena
  const c64* const* kptr;              // 27 FP64 kernel spectra, index (dz+1)*9+(dy+1)*3+dx+1
};

// A near tile: 2 x RZ rows (y0 + ry, z0 + rz), row r = ry + 2 rz, of up to 4 targets along x at
// x0 = 4 wx (RZ = 2 or 4).  The 4 x (RZ + 2) source rows (y0 - 1 + qy, z0 - 1 + qz),
// q = qy + 4 qz, cover the 27 neighbours of every target of the tile; a workgroup stages them
// in LDS once per frequency chunk.
constexpr int kTileW = 4;                 // targets per tile row
constexpr int kTileRowsMax = 8;           // 2 x RZ rows
constexpr int kTileSrcRowsMax = 24;       // 4 x (RZ + 2) source rows
template <typename T> struct NearTile {
  int32_t tgt[kTileRowsMax][kMacL];    // target super slots (-1: none), first kTileW used
  int32_t src[kTileSrcRowsMax * (kTileW + 2)];   // source super slot of row q at x0 - 1 + s:
                                       // [q * 6 + s] (the zero slot where absent)
  uint32_t src_mask;                   // bit q: source row q holds a source
  uint32_t row_mask;                   // bit r: row r holds a target
  int32_t zero;                        // the zero slot (not loaded: staged as zeros)
  int32_t rz;                          // rows along z: 2 or 4
  const cpx<T>* fhat;
  cpx<T>* uhat;
  const cpx<T>* const* kptr;           // 27 kernel spectra in the storage type, index
                                       // (dz+1)*9+(dy+1)*3+dx+1
};

// A compact near tile (FP32, pipelined form): the rows and source rows of a NearTile, but only
// the source spectra that exist are staged: entry e < nreal holds slot src[e], and
// loff[q * 6 + s] is the LDS element offset (entry * 64) of source row q at x0 - 1 + s, that of
// the all-zero entry NC where the source is absent.  NC, the staging capacity, comes with the
// launch mode (near_ctile_cap): tiles with more source super-blocks take the one-chunk form.
constexpr int kCTileCapMax = 48;
template <typename T> struct NearCTile {
  int32_t tgt[kTileRowsMax][kMacL];    // target super slots (-1: none), first kTileW used
  int32_t src[kCTileCapMax];           // slots of the staged entries (the zero slot past nreal)
  uint32_t loff[kTileSrcRowsMax * (kTileW + 2)];
  uint32_t src_mask;                   // bit q: source row q holds a source
  uint32_t row_mask;                   // bit r: row r holds a target
  int32_t nreal;                       // staged entries
  int32_t rz;                          // rows along z: 2 or 4
  int32_t zero;                        // the zero slot (an all-zero spectrum)
  int32_t edges;                       // 1: some source row holds a source at x0 - 1 or x0 + 4
  const cpx<T>* fhat;                  // source super-block slots (spectra, or line-major planes)
  cpx<T>* uhat;                        // target super-block slots
  const cpx<T>* const* kptr;           // as in NearTile
  const cpx<T>* ktr;                   // fused form: kernel columns [14][line][kz] (storage type)
};
constexpr int kNearRunMin = 2, kNearRunMax = 8;   // frequency chunks a pipelined workgroup walks

// TC: element type of the child level, TP: of the parent level (they differ where an FP32
// base level meets FP64 coarse levels).
template <typename TC, typename TP> struct AnterpItem {
  TP* dst;               // parent block, overwritten with sum_c R_c child_c
  const TC* child[8];    // octant c = cx + 2 cy + 4 cz (nullptr: see child_in)
  int64_t child_in[8];   // where child is null: offset of the child in WorkSet::in (FP64
                         // children only), -1: absent
};

// child block pointer of a work item: its own pointer, else (FP64 children) the pass's input
template <typename TC>
__device__ __forceinline__ const TC* child_ptr(const TC* c, int64_t in_off, const double* in) {
  if constexpr (sizeof(TC) == sizeof(double)) {
    if (!c && in_off >= 0) return (const TC*)(in + in_off);
  }
  return c;
}
template <typename TC, typename TP> struct InterpItem {
  TC* child;             // child block: child (+)= J_c parent
  const TP* parent;
  int32_t octant;
  int32_t accumulate;    // 1: add to the child's own level-interaction result, 0: overwrite
};
// Fields that come from the solve pass's input / output are addressed by offsets into
// WorkSet::in / WorkSet::out; plan-owned buffers by pointers.
template <typename T> struct CombineItem {
  double* dst_d;         // plan buffer destination, or, if null,
  int64_t dst_out;       // offset into WorkSet::out
  const T* v;            // level field (nullptr: zero)
  const T* far;          // interpolated coarse-level field, kept apart from v (nullptr: zero)
  const double* base;    // added field (nullptr: zero)
  double scale;          // dst = base + scale * (v + far)
};
template <typename T> struct ConvertItem {
  T* dst;
  const double* src;     // plan buffer, or nullptr: WorkSet::in + src_in
  int64_t src_in;
};
struct CoarsenItem {
  double* dst;           // non-leaf block source = mean of the 2x2x2 child cells
  const double* child[8];
  int64_t child_in[8];   // used where child[c] is null: WorkSet::in + child_in[c]
};
// The interpolated coarse field and the leaf-only field stay in FP64 in both precisions: the
// correction takes their 7-point Laplacian scaled by h^-2, which would turn FP32 rounding of the
// stored values into a source error that the next convolution spreads over the whole level.
struct RefineItem {
  double* jw;            // child block values of J^{l-1} w^{l-1}
  const double* parent_w;  // parent's leaf-only field
  int32_t octant;
  int32_t pad;
};
template <typename T> struct CorrectItem {
  T* g;                  // corrected source g = f - h^-2 L(Jw), rounded to T
  const double* f;       // (coarsened) level source, or nullptr: WorkSet::in + f_in
  int64_t f_in;
  const double* jw;      // own Jw
  const double* nbr[6];  // neighbour blocks' Jw (-x,+x,-y,+y,-z,+z), nullptr: ghost from parent
  const double* parent_w;  // parent field for ghost values
  int32_t octant;
  int32_t pad;
  double inv_h2;
};
struct ResidualItem {
  double* r;             // r = f - h^-2 L u where all 6 neighbours exist, 0 elsewhere (or null)
  float* conv;           // the same rounded to FP32 (the correction pass's base-level source
                         // of a leaf block, written here instead of by a separate convert), or null
  int64_t off;           // block offset of f (in WorkSet::in) and u (in WorkSet::out)
  int64_t nbr_off[6];    // same-level neighbour blocks of u in WorkSet::out (-1: absent)
  double inv_h2;
  int32_t leaf;          // 0: whole block r = 0
  int32_t pad;
};
constexpr int kResidualSlabs = 4;       // workgroups (z-slabs) per block of the residual

// forward operators of the per-level lattice (7-point Laplacian, gradient, curl): one per block
struct OpItem {
  int64_t off;           // block offset in every component array
  int64_t nbr_off[6];    // same-level blocks across faces (-x,+x,-y,+y,-z,+z) (-1: absent)
  int64_t par_off;       // the parent block (ghost values at level boundaries), -1 on level 0
  double inv_h;          // 2^level: inverse spacing in base cells
  int32_t leaf;          // 0: every output cell of the block is 0
  int32_t octant;        // the block's octant in its parent, cx + 2 cy + 4 cz
};

// ----------------------------------------------------------------------------- launchers
// workspace binding: img[idx[i]] += delta for i < n (8-byte words); fill of up to kFillMax
// device ranges (16-byte multiples at 16-byte aligned offsets from base) with a 32-bit pattern
constexpr int kFillMax = 16;
struct FillRanges {
  int32_t n;
  int32_t pad;
  int64_t off[kFillMax];
  int64_t bytes[kFillMax];
};
hipError_t launch_relocate(uint64_t* img, const uint32_t* idx, int64_t n, uint64_t delta, hipStream_t st);
hipError_t launch_fill(uint8_t* base, const FillRanges& r, uint32_t pattern, hipStream_t st);
// one adaptation step of a block layout by the refinement criterion (layout.hip); device arrays
// in and out, *n_out = blocks of the new layout (hipErrorOutOfMemory if above cap)
hipError_t layout_adapt(const int32_t* blocks, const int32_t* levels, int64_t n, int nb, const double* field,
                        int n_levels, double alpha, int32_t* out_blocks, int32_t* out_levels, int64_t cap,
                        int64_t* n_out, hipStream_t st);
int quad_nodes();
// op 0: Laplacian (1 -> 1 component), 1: gradient (1 -> 3), 2: curl (3 -> 3); components of
// u and out are n * nb^3 apart; w3: the quadratic refinement table of the ghost values
hipError_t launch_fwd_op(int nb, int op, const OpItem* items, int64_t n, const double* u, double* out,
                         const double* w3, hipStream_t st);
hipError_t launch_green_table(double* d_cube, double* d_nodes, double* d_wts, const int16_t* d_tri,
                              int ntri, hipStream_t st);
hipError_t launch_green_eval(const int32_t* d_n, int64_t m, const double* d_cube, double* d_out,
                             hipStream_t st);
hipError_t launch_kernel_spectra(int nb, int nspec, const int32_t* d_sd, const double* d_cube,
                                 double* d_real, c64* d_tmp, c64* d_out64, c32* d_out32,
                                 hipStream_t st);

// Each launcher takes a set table whose WorkSet.items point at device arrays of the item type.
// The launcher fills wg_begin from the counts and returns the number of workgroups used.
template <typename T> hipError_t launch_fft_fwd(int nb, SetTable& t, hipStream_t st);
template <typename T> hipError_t launch_fft_inv(int nb, SetTable& t, hipStream_t st);
template <typename T> hipError_t launch_mac(int nb, SetTable& t, hipStream_t st, int mode = 0);
// candidate launch shapes for the autotuner, the planner's default first (FP64: shared sources)
constexpr int kMacModes32[4] = {1, 2, 4, 8};
constexpr int kMacModes64[4] = {1, 2, 6, 8};
constexpr int kMacDefault64 = 8;                 // shared sources (FP64 steps, coarse levels)
template <typename TC, typename TP> hipError_t launch_anterp(int nb, SetTable& t, hipStream_t st);  // ws.w = W
template <typename TC, typename TP> hipError_t launch_interp(int nb, SetTable& t, hipStream_t st);  // ws.w = W
template <typename T> hipError_t launch_combine(int nb, SetTable& t, hipStream_t st);
template <typename T> hipError_t launch_convert(int nb, SetTable& t, hipStream_t st);
hipError_t launch_coarsen(int nb, SetTable& t, hipStream_t st);
hipError_t launch_refine(int nb, SetTable& t, hipStream_t st);                          // ws.w = W3
template <typename T> hipError_t launch_correct(int nb, SetTable& t, hipStream_t st);  // ws.w = W3
hipError_t launch_residual(int nb, SetTable& t, hipStream_t st);
// mode 0: (x, y) pass and z pass through the plane stack [z][line] (spectra for the near MAC);
// mode 1: (x, y) pass only, planes line-major [line][z] (for and from the fused near step)
template <typename T, typename TC> hipError_t launch_super_fwd(int nb, SetTable& t, hipStream_t st, int mode = 0);
template <typename T, typename TC> hipError_t launch_super_inv(int nb, SetTable& t, hipStream_t st, int mode = 0);
// kernel columns for the fused form: out[(h * PLANE + line) * P + kz] = K_h[kz * PLANE + line]
// for the 14 super-block kernels h <= 13 of a set (P = 4 nb, PLANE = P (2 nb + 1))
template <typename T> hipError_t launch_kernel_columns(int nb, const cpx<T>* spectra, cpx<T>* out, hipStream_t st);
// mode: W (2, 4 or 8) for NearRow items; kNearTiled + 4 / + 6 for NearTile items of RZ = 2 / 4;
// NearCTile items (pipelined form, FP32): kNearTiled + 5 / + 7 for RZ = 2 / 4, staging at most
// 36 / 48 source spectra per tile
// Fused form (NearCTile items, FP32 and FP64): kNearFused + 2 / + 4 for RZ = 2 / 4.  The
// super-block transforms of the step's level then take mode 1: the forward (x, y) pass writes the
// planes line-major, [line][z] in the first half of each slot, the fused kernel does the z
// transforms, the MAC and the inverse z transforms per (tile, line), and the inverse (y, x) pass
// reads the line-major target planes.
constexpr int kNearTiled = 16;
constexpr int kNearFused = 40;
constexpr bool near_piped(int mode) { return mode == kNearTiled + 5 || mode == kNearTiled + 7; }
constexpr bool near_fused(int mode) { return mode == kNearFused + 2 || mode == kNearFused + 4; }
constexpr bool near_compact(int mode) { return near_piped(mode) || near_fused(mode); }
constexpr int near_ctile_rz(int mode) { return (mode == kNearTiled + 5 || mode == kNearFused + 2) ? 2 : 4; }
constexpr int near_ctile_cap(int mode) { return near_ctile_rz(mode) == 2 ? 36 : 48; }
template <typename T> hipError_t launch_near_mac(int nb, SetTable& t, hipStream_t st, int mode);

// number of workgroups each item of a kernel needs (for set-table bookkeeping)
inline int64_t assign_wg(SetTable& t, int64_t per_item_num, int64_t per_item_den = 1) {
  int64_t wg = 0;
  for (int i = 0; i < t.n; ++i) {
    t.s[i].wg_begin = wg;
    wg += (t.s[i].count * per_item_num + per_item_den - 1) / per_item_den;
  }
  return wg;
}

}  // namespace lgf
