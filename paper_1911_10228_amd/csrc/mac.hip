// Spectral multiply-accumulate of the level interaction (Sec. 2.1, Algorithm 1 step 2):
//   U_t[k] = sum over the interaction list of t of K_{s, t-src}[k] * F_src[k]
// for every frequency k of the half spectrum.  The list of a target follows from its parity
// (Fig. fmm_regions): its sources are the children of its parent's neighbours, i.e. the offsets
// d = t - src with c_i - 3 <= d_i <= c_i + 2 (c = parity of t); on coarse levels the near region
// |d|_inf <= 1 is excluded, on the base level it is included.
//
// Work unit: a tile of 2x2 sibling target rows (W = 8 targets along x each, or 4 on levels only a
// few blocks wide) and 64 consecutive frequencies (one per lane).  Siblings share their parent's
// neighbours, so the four rows draw from the same 36 source rows.  A wavefront accumulates ROWS
// of the tile's rows (1, 2 or 4): for each source row it holds the W + 6 source spectra of the x
// window in registers and reuses them against the 7 kernel offsets along x and its rows.  The next source row's spectra (and,
// without LDS staging, its kernel spectra) are loaded before the current row's arithmetic, so a
// single wait per source row covers the memory latency.  In FP32 the kernel spectra of the
// level are staged in LDS for the workgroup's 64 frequencies; only offsets d <= 0
// (lexicographically) are stored: the kernel is real and even in every coordinate, so
// K_{-d}[k] = conj(K_d[k]).  All control flow is uniform per wavefront.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <type_traits>

#include "kernels.hpp"

namespace lgf {

namespace {

constexpr int kHalfK = 172;      // offsets with (dz, dy, dx) <= 0 lexicographically: index <= 171

template <typename T> using gptr = const __attribute__((address_space(1))) T*;
template <typename T> using gmut = __attribute__((address_space(1))) T*;
using cptr64 = const __attribute__((address_space(4))) uint64_t*;   // scalar-loadable table

template <typename T> __device__ __forceinline__ cpx<T> gload(gptr<T> base, int64_t i) {
  return {base[2 * i], base[2 * i + 1]};
}

// absent sources point at the arena's all-zero spectrum, so every load is unconditional
template <typename T, int NS>
__device__ __forceinline__ void load_src(cpx<T> (&fs)[NS], const int32_t* __restrict__ sr,
                                         gptr<T> F, int S, int k) {
#pragma unroll
  for (int s = 0; s < NS; ++s) fs[s] = gload<T>(F, (int64_t)sr[s] * S + k);
}

__device__ __forceinline__ int kindex(int r, int jz, int jy, int dxi) {
  const int ry = r & 1, rz = r >> 1;
  return (rz + 5 - jz) * 49 + (ry + 5 - jy) * 7 + dxi;   // (dz+3)*49 + (dy+3)*7 + dx+3
}

// kernel value of offset index h (only h < kHalfK is read: K_{-d}[k] = conj(K_d[k]), so each
// frequency chunk touches 172 kernel spectra instead of 343)
template <typename T>
__device__ __forceinline__ cpx<T> kload(cptr64 kp, int h, int k) {
  const bool mirror = h >= kHalfK;
  cpx<T> v = gload<T>((gptr<T>)kp[mirror ? 342 - h : h], k);
  if (mirror) v.y = -v.y;
  return v;
}

// -v where neg, else v, as an exclusive-or of the sign bit (no select)
__device__ __forceinline__ double flip_sign(double v, bool neg) {
  return __longlong_as_double(__double_as_longlong(v) ^ ((long long)neg << 63));
}

template <typename T, int ROWS>
__device__ __forceinline__ void load_k(cpx<T> (&ks)[ROWS][7], cptr64 kp, int r0, int jz, int jy, int k) {
#pragma unroll
  for (int q = 0; q < ROWS; ++q)
#pragma unroll
    for (int dxi = 0; dxi < 7; ++dxi) ks[q][dxi] = kload<T>(kp, kindex(r0 + q, jz, jy, dxi), k);
}

// accumulate one source row (jz, jy) into target row r (XW targets) with kernel values kv(dxi).
// INNER: the row's sources lie within the targets' x extent (x0 .. x0 + XW - 1), the other
// window entries being the all-zero spectrum; their products are skipped (and fs[] outside
// XW + 3 .. 3 need not be set), which leaves every sum's remaining terms in the same order.
template <typename T, int XW, bool INNER = false, typename KF>
__device__ __forceinline__ void mac_row(cpx<T> (&acc)[XW], const cpx<T> (&fs)[XW + 6], int r, int jz,
                                        int jy, bool base, KF&& kv) {
  const int ry = r & 1, rz = r >> 1;
  const int dz = rz + 2 - jz, dy = ry + 2 - jy;
  const bool near_zy = dz >= -1 && dz <= 1 && dy >= -1 && dy <= 1;
#pragma unroll
  for (int dxi = 0; dxi < 7; ++dxi) {
    const int dx = dxi - 3;
    if (INNER && (dx <= -XW || dx >= XW)) continue;
    if (!base && near_zy && dx >= -1 && dx <= 1) continue;
    const cpx<T> kk = kv(dxi);
#pragma unroll
    for (int i = 0; i < XW; ++i) {
      const int c = i & 1;
      if (dx < c - 3 || dx > c + 2) continue;
      if (INNER && (i - dx < 0 || i - dx >= XW)) continue;
      cmac(acc[i], kk, fs[i - dx + 3]);
    }
  }
}

// SPLIT = 6: the six waves of a workgroup share one (tile, row group) and take one source-row
// plane jz each; their partial sums are added in a fixed order through LDS (for small levels).
// XW = 8 or 4 targets per row (the tiles' x window; rows of 4 for levels only a few blocks wide).
template <typename T, int WAVES, int ROWS, bool KLDS, int SPLIT, int XW>
__global__ __launch_bounds__(64 * WAVES) void mac_tile_kernel(SetTable sets, int S) {
  constexpr int NS = XW + 6;
  __shared__ cpx<T> klds[KLDS ? kHalfK * 64 : 1];
  __shared__ cpx<T> red[SPLIT > 1 ? (SPLIT - 1) * ROWS * XW * 64 : 1];
  constexpr int UPT = 4 / ROWS;                  // units (row groups) per tile
  constexpr int UPW = WAVES / SPLIT;             // units per workgroup
  const int set = find_set(sets, blockIdx.x);
  const WorkSet& ws = sets.s[set];
  const int64_t local = blockIdx.x - ws.wg_begin;       // wg_begin is a multiple of 8
  const int ngroups = (ws.count * UPT + UPW - 1) / UPW;
  // XCD-aware order: workgroups are dealt to the 8 XCDs round-robin, so all workgroups of one
  // frequency chunk get the same residue mod 8 and share one L2 for that chunk's spectra.
  const int xcd = (int)(local & 7);
  const int64_t j = local >> 3;
  const int chunk = (int)(j / ngroups) * 8 + xcd;
  const int grp = (int)(j % ngroups);
  if (chunk * 64 >= S) return;
  // the wave index is uniform within a wavefront; readfirstlane lets the compiler keep the
  // tile descriptor in scalar registers and branch on it without exec masking
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int k = chunk * 64 + lane;
  const MacTile<T>* tiles = (const MacTile<T>*)ws.items;
  const int unit = grp * UPW + wave / SPLIT;
  const int ti = unit / UPT;
  const int r0 = (unit % UPT) * ROWS;
  const int part = SPLIT > 1 ? wave % SPLIT : 0;
  const bool active = ti < ws.count;
  const MacTile<T>* tile = tiles + (active ? ti : (grp * UPW) / UPT);
  const cptr64 kp = (cptr64)tile->kptr;          // one level (one kernel set) per work set

  if constexpr (KLDS) {
    for (int h = wave; h < kHalfK; h += WAVES) klds[h * 64 + lane] = gload<T>((gptr<T>)kp[h], k);
    __syncthreads();
  }
  if (!active) return;
  const int rmask = tile->row_mask;
  const int mymask = (rmask >> r0) & ((1 << ROWS) - 1);
  if (!mymask) return;           // with SPLIT, all waves of the group take this exit together

  const bool base = tile->flags & 1;
  uint64_t todo = tile->pair_mask;
  if constexpr (SPLIT > 1) todo &= 0x3Full << (6 * part);
  gptr<T> F = (gptr<T>)tile->fhat;

  cpx<T> acc[ROWS][XW];
#pragma unroll
  for (int q = 0; q < ROWS; ++q)
#pragma unroll
    for (int i = 0; i < XW; ++i) acc[q][i] = {T(0), T(0)};

  if (todo) {
    int pj = __builtin_ctzll(todo);
    todo &= todo - 1;
    cpx<T> fs[NS];
    cpx<T> ks[KLDS ? 1 : ROWS][7];
    load_src<T, NS>(fs, tile->src[pj], F, S, k);
    if constexpr (!KLDS) load_k<T, ROWS>(ks, kp, r0, pj / 6, pj % 6, k);
    for (;;) {
      // the next source row's loads are issued unconditionally (the last iteration reloads the
      // current row), so every iteration issues the same loads and the waits for the current
      // row leave the next row's loads in flight (the vector memory counter retires in order)
      const bool more = todo != 0;
      const int pn = more ? __builtin_ctzll(todo) : pj;
      todo &= todo - 1;
      cpx<T> fn[NS];
      cpx<T> kn[KLDS ? 1 : ROWS][7];
      load_src<T, NS>(fn, tile->src[pn], F, S, k);
      if constexpr (!KLDS) load_k<T, ROWS>(kn, kp, r0, pn / 6, pn % 6, k);
      const int jz = pj / 6, jy = pj % 6;
#pragma unroll
      for (int q = 0; q < ROWS; ++q) {
        if (!((mymask >> q) & 1)) continue;
        const int r = r0 + q;
        if constexpr (KLDS) {
          mac_row<T, XW>(acc[q], fs, r, jz, jy, base, [&](int dxi) {
            const int idx = kindex(r, jz, jy, dxi);
            const bool mirror = idx >= kHalfK;
            cpx<T> kv = klds[(mirror ? 342 - idx : idx) * 64 + lane];
            if (mirror) kv.y = -kv.y;
            return kv;
          });
        } else {
          mac_row<T, XW>(acc[q], fs, r, jz, jy, base, [&](int dxi) { return ks[q][dxi]; });
        }
      }
      if (!more) break;
#pragma unroll
      for (int s = 0; s < NS; ++s) fs[s] = fn[s];
      if constexpr (!KLDS) {
#pragma unroll
        for (int q = 0; q < ROWS; ++q)
#pragma unroll
          for (int d = 0; d < 7; ++d) ks[q][d] = kn[q][d];
      }
      pj = pn;
    }
  }
  if constexpr (SPLIT > 1) {
    // ordered reduction of the partial sums: wave 0 adds parts 1..SPLIT-1 in turn
    static_assert(WAVES == SPLIT, "split mode: one (tile, row group) per workgroup");
    if (part > 0) {
#pragma unroll
      for (int q = 0; q < ROWS; ++q)
#pragma unroll
        for (int i = 0; i < XW; ++i) red[(((part - 1) * ROWS + q) * XW + i) * 64 + lane] = acc[q][i];
    }
    __syncthreads();
    if (part > 0) return;
    for (int p = 1; p < SPLIT; ++p)
#pragma unroll
      for (int q = 0; q < ROWS; ++q)
#pragma unroll
        for (int i = 0; i < XW; ++i) {
          const cpx<T> v = red[(((p - 1) * ROWS + q) * XW + i) * 64 + lane];
          acc[q][i].x += v.x;
          acc[q][i].y += v.y;
        }
  }
  gmut<T> U = (gmut<T>)tile->uhat;
#pragma unroll
  for (int q = 0; q < ROWS; ++q)
#pragma unroll
    for (int i = 0; i < XW; ++i) {
      const int t = tile->tgt[r0 + q][i];
      if (t >= 0) {
        U[2 * ((int64_t)t * S + k)] = acc[q][i].x;
        U[2 * ((int64_t)t * S + k) + 1] = acc[q][i].y;
      }
    }
}

// Shared-source form (kernel spectra from memory): the tile's 4 wavefronts (one target row each)
// walk the tile's source rows together.  Each source row's XW + 6 spectra are loaded once per
// workgroup, spread over the wavefronts, into one of two LDS buffers, and every wavefront reads
// them from there; its 7 kernel values come from memory.  The next source row's spectra and
// kernel values are loaded while the current row is applied, one barrier per source row
// (double buffering: a buffer is rewritten only after the barrier that follows its last reads).
template <typename T, int XW>
__global__ __launch_bounds__(256) void mac_shared_kernel(SetTable sets, int S) {
  constexpr int NS = XW + 6;
  constexpr int PW = (NS + 3) / 4;               // staged spectra per wavefront and source row
  __shared__ cpx<T> sb[2][NS * 64];
  const int set = find_set(sets, blockIdx.x);
  const WorkSet& ws = sets.s[set];
  const int64_t local = blockIdx.x - ws.wg_begin;       // wg_begin is a multiple of 8
  const int ntiles = ws.count;
  const int xcd = (int)(local & 7);
  const int64_t j = local >> 3;
  const int chunk = (int)(j / ntiles) * 8 + xcd;
  const int ti = (int)(j % ntiles);
  if (chunk * 64 >= S) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int k = chunk * 64 + lane;
  const MacTile<T>* tile = (const MacTile<T>*)ws.items + ti;
  const cptr64 kp = (cptr64)tile->kptr;
  gptr<T> F = (gptr<T>)tile->fhat;
  const int r = wave;
  const bool row = (tile->row_mask >> r) & 1;
  const bool base = tile->flags & 1;
  uint64_t todo = tile->pair_mask;
  cpx<T> acc[XW];
#pragma unroll
  for (int i = 0; i < XW; ++i) acc[i] = {T(0), T(0)};
  if (todo) {
    // staged entries of this wavefront: e = wave + 4 q (q < PW, e < NS); kernel values of row r
    int pj = __builtin_ctzll(todo);
    todo &= todo - 1;
    cpx<T> st[PW], ks[7];
#pragma unroll
    for (int q = 0; q < PW; ++q) {
      const int e = wave + 4 * q;
      if (e < NS) st[q] = gload<T>(F, (int64_t)tile->src[pj][e] * S + k);
    }
#pragma unroll
    for (int d = 0; d < 7; ++d) ks[d] = kload<T>(kp, kindex(r, pj / 6, pj % 6, d), k);
    int buf = 0;
    for (;;) {
#pragma unroll
      for (int q = 0; q < PW; ++q) {
        const int e = wave + 4 * q;
        if (e < NS) sb[buf][e * 64 + lane] = st[q];
      }
      __syncthreads();
      // next source row (the last iteration reloads the current one: same loads every time)
      const bool more = todo != 0;
      const int pn = more ? __builtin_ctzll(todo) : pj;
      todo &= todo - 1;
#pragma unroll
      for (int q = 0; q < PW; ++q) {
        const int e = wave + 4 * q;
        if (e < NS) st[q] = gload<T>(F, (int64_t)tile->src[pn][e] * S + k);
      }
      cpx<T> kn[7];
#pragma unroll
      for (int d = 0; d < 7; ++d) kn[d] = kload<T>(kp, kindex(r, pn / 6, pn % 6, d), k);
      if (row) {
        cpx<T> fs[NS];
#pragma unroll
        for (int e = 0; e < NS; ++e) fs[e] = sb[buf][e * 64 + lane];
        mac_row<T, XW>(acc, fs, r, pj / 6, pj % 6, base, [&](int dxi) { return ks[dxi]; });
      }
      if (!more) break;
#pragma unroll
      for (int d = 0; d < 7; ++d) ks[d] = kn[d];
      pj = pn;
      buf ^= 1;
    }
  }
  if (!row) return;
  gmut<T> U = (gmut<T>)tile->uhat;
#pragma unroll
  for (int i = 0; i < XW; ++i) {
    const int t = tile->tgt[r][i];
    if (t >= 0) {
      U[2 * ((int64_t)t * S + k)] = acc[i].x;
      U[2 * ((int64_t)t * S + k) + 1] = acc[i].y;
    }
  }
}

// LDS form (coarse levels with rows of 4 targets whose source slots lie within kMacLdsSrc of
// each other, i.e. small levels): a workgroup takes one chunk of 16 frequencies and up to 4 tiles
// (one per wavefront; lane = (row of the tile, frequency)).  It first stages, with every load
// issued at once, the chunk's kernel values (the 172 offsets d <= 0 lexicographically: K_{-d} =
// conj K_d; in FP64 also d = (0, 0, 1..3) as conjugates of (0, 0, -1..-3)) and the
// chunk's values of the step's source spectra (the slots [src_lo, src_lo + src_n), plus one
// zero entry for absent sources) and the tiles' source slot tables (as LDS entry indices), then
// walks the source rows from LDS only: one memory round trip per workgroup instead of one per
// source row, and every kernel spectrum read once per chunk and group of tiles.  Groups of 4
// tiles of one chunk run on one XCD (they read the same kernel values).  With the three extra
// entries, the 7 offsets along x of one (target row, source row) pair are either all stored or
// all conjugates of stored ones (d > 0 lexicographically for every dx iff (dz, dy) > 0), so a
// lane decides that once per source row instead of once per offset (level 1 of the 8^3 layout
// of 16^3 blocks, FP64: 47.2 -> 44.2 us).  FP32 decides per offset: with the extra entries its workgroups ran slower (30.0 ->
// 31.7-32.5 us; they take it from 31.8 to 32.2 KB of LDS, near the share of five per CU).
constexpr int kLdsF = 16;
template <typename T> constexpr int kLdsK = sizeof(T) == 8 ? kHalfK + 3 : kHalfK;
template <typename T>
__global__ __launch_bounds__(256) void mac_lds_kernel(SetTable sets, int S) {
  constexpr int XW = kMacL / 2, NS = XW + 6, F = kLdsF, NSRC = kMacLdsSrc;
  constexpr int NKE = kLdsK<T>;
  __shared__ cpx<T> KL[NKE * F];                  // kernel values, [h][f]
  __shared__ cpx<T> SL[(NSRC + 1) * F];           // source values, [entry][f]; entry NSRC: zeros
  __shared__ uint8_t IX[4][36][NS];               // LDS entry of tile w's source row j, slot s
  const int set = find_set(sets, blockIdx.x);
  const WorkSet& ws = sets.s[set];
  const int64_t local = blockIdx.x - ws.wg_begin;      // wg_begin is a multiple of 8
  const int ngroups = (ws.count + 3) / 4;
  const int64_t jw = local >> 3;
  const int chunk = (int)(jw / ngroups) * 8 + (int)(local & 7);
  const int grp = (int)(jw % ngroups);
  if (chunk * F >= S) return;
  const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const MacTile<T>* tiles = (const MacTile<T>*)ws.items + 4 * grp;
  const int ntile = min(4, ws.count - 4 * grp);
  const int lo = tiles[0].src_lo, n = tiles[0].src_n;
  const cptr64 kp = (cptr64)tiles[0].kptr;
  const gptr<T> Fh = (gptr<T>)tiles[0].fhat;
  // stage: kernel values, source values, slot tables (all loads issued before the first store)
  constexpr int NK = (NKE * F + 255) / 256, NV = ((NSRC + 1) * F + 255) / 256;
  cpx<T> kv[NK], sv[NV];
#pragma unroll
  for (int j = 0; j < NK; ++j) {
    const int i = tid + 256 * j;
    const int h = i / F;                          // h >= kHalfK: conj K of offset 342 - h
    if (i < NKE * F) kv[j] = gload<T>((gptr<T>)kp[h < kHalfK ? h : 342 - h], (int64_t)chunk * F + i % F);
  }
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    const int i = tid + 256 * j, e = i / F;
    sv[j] = cpx<T>{T(0), T(0)};
    if (e < n) sv[j] = gload<T>(Fh, (int64_t)(lo + e) * S + (int64_t)chunk * F + i % F);
  }
  constexpr int NI = (4 * 36 * NS + 255) / 256;
  int sl[NI];
#pragma unroll
  for (int m = 0; m < NI; ++m) {
    const int i = tid + 256 * m, w = i / (36 * NS), r = i % (36 * NS);
    sl[m] = (i < 4 * 36 * NS && w < ntile) ? tiles[w].src[r / NS][r % NS] : lo - 1;
  }
#pragma unroll
  for (int j = 0; j < NK; ++j) {
    const int i = tid + 256 * j;
    if (i < NKE * F) KL[i] = i < kHalfK * F ? kv[j] : cpx<T>{kv[j].x, -kv[j].y};
  }
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    const int i = tid + 256 * j;
    if (i < (NSRC + 1) * F) SL[i] = sv[j];
  }
#pragma unroll
  for (int m = 0; m < NI; ++m) {
    const int i = tid + 256 * m;
    const unsigned d = (unsigned)(sl[m] - lo);
    if (i < 4 * 36 * NS) (&IX[0][0][0])[i] = d < (unsigned)n ? (uint8_t)d : (uint8_t)NSRC;
  }
  __syncthreads();
  if (wave >= ntile) return;
  const MacTile<T>& tile = tiles[wave];
  const int f = lane % F, r = lane / F;           // row r of the tile, frequency chunk F + f
  const bool base = tile.flags & 1;
  cpx<T> acc[XW];
#pragma unroll
  for (int i = 0; i < XW; ++i) acc[i] = {T(0), T(0)};
  auto walk = [&](auto inner) {
    constexpr bool INNER = decltype(inner)::value;
    auto in_window = [](int q) { return !INNER || (q >= 3 && q < 3 + XW); };
    // Pipelined: while a row's products run, the next row's source and kernel values and the
    // slot-table entries of the row after it are in flight (LDS reads complete in issue order,
    // so each wait leaves the younger reads outstanding).  Past the last row the walk re-reads
    // that row, so every step issues the same reads.
    const int n = __builtin_popcountll(tile.pair_mask);
    uint64_t todo = tile.pair_mask;
    auto next = [&](int prev) {
      if (!todo) return prev;
      const int p = __builtin_ctzll(todo);
      todo &= todo - 1;
      return p;
    };
    auto read_ix = [&](int pj, uint8_t (&x)[NS]) {
#pragma unroll
      for (int q = 0; q < NS; ++q)
        if (in_window(q)) x[q] = IX[wave][pj][q];
    };
    // the row's source values and its 7 kernel values along x (FP64: one mirror decision per
    // row; FP32: one per offset)
    auto read_vals = [&](int pj, const uint8_t (&x)[NS], cpx<T> (&fs)[NS], cpx<T> (&kv)[7]) {
#pragma unroll
      for (int q = 0; q < NS; ++q)
        if (in_window(q)) fs[q] = SL[x[q] * F + f];
      const int jz = pj / 6, jy = pj % 6;
      if constexpr (sizeof(T) == 8) {
        const int dz = (r >> 1) + 2 - jz, dy = (r & 1) + 2 - jy;
        const bool conj = dz > 0 || (dz == 0 && dy > 0);
        const int h0 = kindex(r, jz, jy, 0);
        const int kb = (conj ? 342 - h0 : h0) * F + f, ks = conj ? -F : F;
#pragma unroll
        for (int d = 0; d < 7; ++d) {
          kv[d] = KL[kb + ks * d];
          kv[d].y = flip_sign(kv[d].y, conj);
        }
      } else {
#pragma unroll
        for (int d = 0; d < 7; ++d) {
          const int h = kindex(r, jz, jy, d);
          const bool mirror = h >= kHalfK;
          kv[d] = KL[(mirror ? 342 - h : h) * F + f];
          if (mirror) kv[d].y = -kv[d].y;
        }
      }
    };
    if (n == 0) return;
    // two register sets in turn (no copies between iterations)
    int pa = next(-1), pb = next(pa);
    uint8_t xa[NS], xb[NS];
    cpx<T> fa[NS], ka[7], fb[NS], kb[7];
    read_ix(pa, xa);
    read_vals(pa, xa, fa, ka);
    read_ix(pb, xb);
    for (int i = 0; i < n; i += 2) {
      const int pc = next(pb);
      read_vals(pb, xb, fb, kb);
      read_ix(pc, xa);
      mac_row<T, XW, INNER>(acc, fa, r, pa / 6, pa % 6, base, [&](int dxi) { return ka[dxi]; });
      if (i + 1 >= n) break;
      const int pd = next(pc);
      read_vals(pc, xa, fa, ka);
      read_ix(pd, xb);
      mac_row<T, XW, INNER>(acc, fb, r, pb / 6, pb % 6, base, [&](int dxi) { return kb[dxi]; });
      pa = pc;
      pb = pd;
    }
  };
  if (tile.flags & 2) walk(std::true_type{});
  else walk(std::false_type{});
  if (!((tile.row_mask >> r) & 1)) return;
  gmut<T> U = (gmut<T>)tile.uhat;
  const int64_t k = (int64_t)chunk * F + f;
#pragma unroll
  for (int i = 0; i < XW; ++i) {
    const int t = tile.tgt[r][i];
    if (t >= 0) {
      U[2 * ((int64_t)t * S + k)] = acc[i].x;
      U[2 * ((int64_t)t * S + k) + 1] = acc[i].y;
    }
  }
}

template <typename T> hipError_t launch_lds(int S, SetTable& t, hipStream_t st) {
  if (S % kLdsF) return hipErrorInvalidValue;
  const int chunks8 = (S / kLdsF + 7) / 8;
  int64_t wg = 0;
  for (int i = 0; i < t.n; ++i) {
    t.s[i].wg_begin = wg;
    wg += (int64_t)((t.s[i].count + 3) / 4) * chunks8 * 8;
  }
  if (wg == 0) return hipSuccess;
  mac_lds_kernel<T><<<(unsigned)wg, 256, 0, st>>>(t, S);
  return hipGetLastError();
}

template <typename T, int XW> hipError_t launch_shared(int S, SetTable& t, hipStream_t st) {
  const int chunks8 = (S / 64 + 7) / 8;
  int64_t wg = 0;
  for (int i = 0; i < t.n; ++i) {
    t.s[i].wg_begin = wg;
    wg += (int64_t)t.s[i].count * chunks8 * 8;
  }
  if (wg == 0) return hipSuccess;
  mac_shared_kernel<T, XW><<<(unsigned)wg, 256, 0, st>>>(t, S);
  return hipGetLastError();
}

template <typename T, int WAVES, int ROWS, bool KLDS, int SPLIT = 1, int XW = kMacL>
hipError_t launch_tiles(int S, SetTable& t, hipStream_t st) {
  constexpr int UPT = 4 / ROWS, UPW = WAVES / SPLIT;
  static_assert(UPW >= 1 && WAVES % SPLIT == 0, "shape");
  const int chunks8 = (S / 64 + 7) / 8;
  int64_t wg = 0;
  for (int i = 0; i < t.n; ++i) {
    t.s[i].wg_begin = wg;
    wg += (int64_t)((t.s[i].count * UPT + UPW - 1) / UPW) * chunks8 * 8;
  }
  if (wg == 0) return hipSuccess;
  mac_tile_kernel<T, WAVES, ROWS, KLDS, SPLIT, XW><<<(unsigned)wg, 64 * WAVES, 0, st>>>(t, S);
  return hipGetLastError();
}

}  // namespace

// Launch shape (mode): 1 row, 2 pair, 4 tile = rows per wavefront; 6 split = FP64 source rows
// over 6 wavefronts; 0 = default (one row per wavefront; FP32 with the kernel spectra in LDS and
// 16 wavefronts per workgroup, FP64 with the kernel spectra prefetched from memory); 8 shared =
// the tile's rows on 4 wavefronts sharing each source row through LDS, kernel spectra from
// memory (the default on coarse levels: few tiles per frequency chunk cannot amortise staging
// all kernel spectra of a chunk).  Bit
// kMacHalfRows marks tiles whose rows hold 4 targets (set by the planner with the items).  The
// plan's autotuner picks the shape per step; LGF_MAC_MODE = row | pair | tile | split | shared
// overrides it.
int mac_mode_override() {
  static const int m = [] {
    const char* e = std::getenv("LGF_MAC_MODE");
    if (!e) return 0;
    if (!std::strcmp(e, "row")) return 1;
    if (!std::strcmp(e, "pair")) return 2;
    if (!std::strcmp(e, "tile")) return 4;
    if (!std::strcmp(e, "split")) return 6;
    if (!std::strcmp(e, "shared")) return 8;
    return 0;
  }();
  return m;
}

template <typename T> hipError_t launch_mac(int nb, SetTable& t, hipStream_t st, int mode) {
  const int P = 2 * nb;
  const int S = P * P * (nb + 1);          // multiple of 64 for nb in {8, 16}
  if (S % 64) return hipErrorInvalidValue;
  const bool half = mode & kMacHalfRows;
  mode &= kMacHalfRows - 1;
  if (const int o = mac_mode_override()) mode = o;
  if (mode == kMacLds) return half ? launch_lds<T>(S, t, st) : hipErrorInvalidValue;
  if (half) {
    if constexpr (sizeof(T) == 4) {
      if (mode == 8) return launch_shared<T, 4>(S, t, st);
      if (mode == 4) return launch_tiles<T, 16, 4, true, 1, 4>(S, t, st);
      if (mode == 2) return launch_tiles<T, 16, 2, true, 1, 4>(S, t, st);
      return launch_tiles<T, 16, 1, true, 1, 4>(S, t, st);
    } else {
      if (mode == 2) return launch_tiles<T, 4, 2, false, 1, 4>(S, t, st);
      if (mode == 6) return launch_tiles<T, 6, 1, false, 6, 4>(S, t, st);
      if (mode == 8) return launch_shared<T, 4>(S, t, st);
      return launch_tiles<T, 4, 1, false, 1, 4>(S, t, st);
    }
  }
  if constexpr (sizeof(T) == 4) {
    if (mode == 8) return launch_shared<T, kMacL>(S, t, st);
    if (mode == 4) return launch_tiles<T, 16, 4, true>(S, t, st);
    if (mode == 2) return launch_tiles<T, 16, 2, true>(S, t, st);
    return launch_tiles<T, 16, 1, true>(S, t, st);
  } else {
    if (mode == 2) return launch_tiles<T, 4, 2, false>(S, t, st);
    if (mode == 6) return launch_tiles<T, 6, 1, false, 6>(S, t, st);
    if (mode == 8) return launch_shared<T, kMacL>(S, t, st);
    return launch_tiles<T, 4, 1, false>(S, t, st);
  }
}

template hipError_t launch_mac<float>(int, SetTable&, hipStream_t, int);
template hipError_t launch_mac<double>(int, SetTable&, hipStream_t, int);

// ============================================================================= near (super) MAC
// U_P[k] = sum over the 27 super-blocks Q with |P - Q|_inf <= 1 of K_{P-Q}[k] F_Q[k].
// Three forms follow: rows (below), one-chunk tiles and pipelined tiles (further down; the
// planner's choice where a level's tiles fit the pipelined form's staging).
// Rows: one wavefront owns a row of W target super-blocks along x and 64 frequencies.  The source rows
// (dy, dz) that hold sources come in groups of 3; a group's 3 (W + 2) source spectra are loaded
// together while the previous group is applied (3 kernel offsets along x each, kernels from LDS).
// Kernel offsets are numbered h = 9 (dz + 1) + 3 (dy + 1) + dx + 1; only h <= 13 is read: the
// zero-padded kernel block is real and G is even in every coordinate (the unused middle plane is
// zero on both sides), so K_{-d}[k] = conj(K_d[k]), i.e. K_h = conj(K_{26-h}).  The products are formed and summed in FP64 from FP64 kernel
// spectra whatever the storage type T of the super-block spectra: the FP64 multiply-add rate
// equals the unpacked FP32 rate, and the FP64 sum keeps the rounding of the largest
// (low-frequency) terms out of the smooth part of the result.
namespace {

constexpr int kNearHalfK = 14;   // kernel offsets h = 0..13 (the centre and one of each +-d pair)

template <typename T, int NS>
__device__ __forceinline__ void load_group(cpx<T> (&f)[3][NS], const NearRow<T>* row, int g,
                                           gptr<T> F, int S, int k) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int s = 0; s < NS; ++s) f[r][s] = gload<T>(F, (int64_t)row->src[3 * g + r][s] * S + k);
}

template <typename T, int W, int NS>
__device__ __forceinline__ void apply_group(cpx<double> (&acc)[W], const cpx<T> (&f)[3][NS],
                                            uint64_t code, int g, const cpx<double>* kl, int lane) {
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const int pj = (int)((code >> (4 * (3 * g + r))) & 15u);
    cpx<double> fd[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) fd[s] = {double(f[r][s].x), double(f[r][s].y)};
#pragma unroll
    for (int dxi = 0; dxi < 3; ++dxi) {
      const int h = pj * 3 + dxi;
      cpx<double> kv = kl[(h < kNearHalfK ? h : 26 - h) * 64 + lane];
      if (h >= kNearHalfK) kv.y = -kv.y;
#pragma unroll
      for (int i = 0; i < W; ++i) cmac(acc[i], kv, fd[i - dxi + 2]);   // src x = x0 + i - dx
    }
  }
}

template <typename T, int W, int NG>
__device__ __forceinline__ void near_groups(cpx<double> (&acc)[W], const NearRow<T>* row,
                                            uint64_t code, gptr<T> F, int S, int k,
                                            const cpx<double>* kl, int lane) {
  constexpr int NS = W + 2;
  cpx<T> fa[3][NS], fb[3][NS];
  load_group<T, NS>(fa, row, 0, F, S, k);
  if constexpr (NG > 1) load_group<T, NS>(fb, row, 1, F, S, k);
  apply_group<T, W, NS>(acc, fa, code, 0, kl, lane);
  if constexpr (NG > 2) load_group<T, NS>(fa, row, 2, F, S, k);
  if constexpr (NG > 1) apply_group<T, W, NS>(acc, fb, code, 1, kl, lane);
  if constexpr (NG > 2) apply_group<T, W, NS>(acc, fa, code, 2, kl, lane);
}

template <typename T, int W>
__global__ __launch_bounds__(256) void near_mac_kernel(SetTable sets, int S) {
  constexpr int NS = W + 2;
  __shared__ cpx<double> kl[kNearHalfK * 64];
  const int set = find_set(sets, blockIdx.x);
  const WorkSet& ws = sets.s[set];
  const int64_t local = blockIdx.x - ws.wg_begin;       // wg_begin is a multiple of 8
  const int ngroups = (ws.count + 3) / 4;
  const int xcd = (int)(local & 7);
  const int64_t j = local >> 3;
  const int chunk = (int)(j / ngroups) * 8 + xcd;
  const int grp = (int)(j % ngroups);
  if (chunk * 64 >= S) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int k = chunk * 64 + lane;
  const NearRow<T>* rows = (const NearRow<T>*)ws.items;
  const int ri = grp * 4 + wave;
  const bool active = ri < ws.count;
  const NearRow<T>* row = rows + (active ? ri : grp * 4);
  const cptr64 kp = (cptr64)row->kptr;
  for (int h = wave; h < kNearHalfK; h += 4) kl[h * 64 + lane] = gload<double>((gptr<double>)kp[h], k);
  __syncthreads();
  if (!active) return;

  gptr<T> F = (gptr<T>)row->fhat;
  cpx<double> acc[W];
#pragma unroll
  for (int i = 0; i < W; ++i) acc[i] = {0.0, 0.0};
  const int ng = row->ngroups;
  const uint64_t code = row->pj_code;
  // straight-line code per group count, so that every wait for a group's loads leaves the next
  // group's loads in flight (the vector memory counter retires in order)
  if (ng == 3) near_groups<T, W, 3>(acc, row, code, F, S, k, kl, lane);
  else if (ng == 2) near_groups<T, W, 2>(acc, row, code, F, S, k, kl, lane);
  else if (ng == 1) near_groups<T, W, 1>(acc, row, code, F, S, k, kl, lane);
  gmut<T> U = (gmut<T>)row->uhat;
#pragma unroll
  for (int i = 0; i < W; ++i) {
    const int t = row->tgt[i];
    if (t >= 0) {
      U[2 * ((int64_t)t * S + k)] = T(acc[i].x);
      U[2 * ((int64_t)t * S + k) + 1] = T(acc[i].y);
    }
  }
}

// Tiled form: one workgroup of 2 RZ wavefronts (one per target row) per (tile, frequency chunk);
// the 4 (RZ + 2) source rows of the tile ((W + 2) spectra each, 64 frequencies) are staged in LDS
// with all loads of a wavefront in flight together, and each wavefront holds the 14 kernel
// values h <= 13 of its frequency in registers (the others are their conjugates).  Each
// wavefront then applies its row's 9 source rows from LDS, in the storage type (the planner uses
// tiles for FP32 spectra on single-level layouts, where defect correction removes FP32 error:
// an FP64 sum there changed nothing measurable).  Compared with one wavefront per row loading
// its own 9 source rows, each source spectrum chunk is read from L2 once per tile instead of up
// to 4 times; taller tiles (RZ = 4) stage fewer spectra per row, in more LDS per workgroup.
template <typename T, int W, int RZ>
__global__ __launch_bounds__(128 * RZ) void near_tile_kernel(SetTable sets, int S) {
  static_assert(W == kTileW, "tile rows hold kTileW targets");
  constexpr int WAVES = 2 * RZ;                    // one per target row
  constexpr int NS = W + 2;
  constexpr int NE = 4 * (RZ + 2) * NS;            // staged spectra per tile
  constexpr int PER_WAVE = NE / WAVES;
  static_assert(NE % WAVES == 0 && 4 * (RZ + 2) <= kTileSrcRowsMax, "tile entries split evenly");
  __shared__ cpx<T> fl[NE * 64];
  const int set = find_set(sets, blockIdx.x);
  const WorkSet& ws = sets.s[set];
  const int64_t local = blockIdx.x - ws.wg_begin;       // wg_begin is a multiple of 8
  const int ntiles = ws.count;
  const int xcd = (int)(local & 7);
  const int64_t j = local >> 3;
  const int chunk = (int)(j / ntiles) * 8 + xcd;
  const int ti = (int)(j % ntiles);
  if (chunk * 64 >= S) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int k = chunk * 64 + lane;
  const NearTile<T>* tile = (const NearTile<T>*)ws.items + ti;
  gptr<T> F = (gptr<T>)tile->fhat;
  const uint32_t smask = tile->src_mask;
  const int r = wave;
  const int ry = r & 1, rz = r >> 1;
  const bool has_row = (tile->row_mask >> r) & 1u;
  {
    // each wavefront stages a contiguous run of entries: one wide scalar load of their slots,
    // then the vector loads back to back; absent sources (the zero slot) are staged as zeros
    // without a load
    static_assert(PER_WAVE <= 64, "one slot per lane");
    const int32_t* sl = tile->src + wave * PER_WAVE;
    const int zero = tile->zero;
    // one vector load of the wavefront's slot list, then each slot broadcast from its lane
    // (scalar loads inside the branches below would each wait for their own round trip)
    const int myslot = lane < PER_WAVE ? sl[lane] : zero;
    cpx<T> v[PER_WAVE];
#pragma unroll
    for (int e = 0; e < PER_WAVE; ++e) {
      const int slot = __builtin_amdgcn_readlane(myslot, e);
      v[e] = slot != zero ? gload<T>(F, (int64_t)slot * S + k) : cpx<T>{T(0), T(0)};
    }
#pragma unroll
    for (int e = 0; e < PER_WAVE; ++e) fl[(wave * PER_WAVE + e) * 64 + lane] = v[e];
  }
  // the kernel values h <= 13 of this lane's frequency (unconditional: the scalar loads of the
  // pointer table then batch)
  const cptr64 kp = (cptr64)tile->kptr;
  cpx<T> kv[kNearHalfK];
#pragma unroll
  for (int h = 0; h < kNearHalfK; ++h) kv[h] = gload<T>((gptr<T>)kp[h], k);
  __syncthreads();
  if (!has_row) return;
  cpx<T> acc[W];
#pragma unroll
  for (int i = 0; i < W; ++i) acc[i] = {T(0), T(0)};
#pragma unroll
  for (int pj = 0; pj < 9; ++pj) {
    const int dz = pj / 3 - 1, dy = pj % 3 - 1;
    const int q = (ry + 1 - dy) + 4 * (rz + 1 - dz);
    if (!((smask >> q) & 1u)) continue;
    cpx<T> fd[NS];
#pragma unroll
    for (int s2 = 0; s2 < NS; ++s2) fd[s2] = fl[(q * NS + s2) * 64 + lane];
#pragma unroll
    for (int dxi = 0; dxi < 3; ++dxi) {
      const int h = pj * 3 + dxi;
      const cpx<T> kk = h < kNearHalfK ? kv[h] : cpx<T>{kv[26 - h].x, -kv[26 - h].y};
#pragma unroll
      for (int i = 0; i < W; ++i) cmac(acc[i], kk, fd[i - dxi + 2]);   // src x = x0 + i - dx
    }
  }
  gmut<T> U = (gmut<T>)tile->uhat;
#pragma unroll
  for (int i = 0; i < W; ++i) {
    const int t = tile->tgt[r][i];
    if (t >= 0) {
      U[2 * ((int64_t)t * S + k)] = T(acc[i].x);
      U[2 * ((int64_t)t * S + k) + 1] = T(acc[i].y);
    }
  }
}

// Pipelined tiled form: a workgroup walks a run of RUN consecutive frequency
// chunks for one compact tile.  The next chunk's source and kernel spectra are copied
// straight from memory into the other of two LDS buffers (global_load_lds: nothing in flight in
// registers) while the current chunk is applied, so loads and arithmetic overlap inside each
// workgroup; in the one-chunk form every resident workgroup loads, then computes, in step with
// the others.  Only the source spectra that exist are staged (NC entries at most, one all-zero
// entry for the absent ones), and the 14 kernel values come from LDS as well.
template <typename T, int RZ, int NC>
__global__ __launch_bounds__(128 * RZ) void near_pipe_kernel(SetTable sets, int S, int RUN) {
  constexpr int W = kTileW, WAVES = 2 * RZ, NS = W + 2;
  constexpr int EPC = 16 / (int)sizeof(cpx<T>);  // entries per 16-byte-per-lane copy: 2 (FP32), 1
  constexpr int LPE = 64 / EPC;                  // lanes per entry
  constexpr int KE = NC + 1;                     // first kernel entry (entry NC: all zeros)
  constexpr int NE = NC + 16;                    // entries per buffer: NC, zero, 14 kernels, spare
  static_assert(NC % 2 == 0 && NC <= kCTileCapMax, "FP32 entries are copied in pairs");
  // two separate LDS objects, each use naming one statically, so that the compiler can tell
  // the copies into one buffer from the reads of the other and does not wait for the copies
  __shared__ cpx<T> fa[NE * 64];
  __shared__ cpx<T> fz[NE * 64];
  const int set = find_set(sets, blockIdx.x);
  const WorkSet& ws = sets.s[set];
  const int64_t local = blockIdx.x - ws.wg_begin;       // wg_begin is a multiple of 8
  const int ntiles = ws.count;
  const int xcd = (int)(local & 7);
  const int64_t j = local >> 3;
  const int run = (int)(j / ntiles) * 8 + xcd;           // all tiles of a run on one XCD
  const int ti = (int)(j % ntiles);
  const int nchunks = S / 64;
  const int c0 = run * RUN;
  if (c0 >= nchunks) return;
  const int nrun = min(RUN, nchunks - c0);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  // the tile through the constant address space: every field read is a scalar load, so the
  // only vector-memory operations in flight are the copies and stores (a wait for a vector load
  // of tile data would also wait for the copies of the next chunk)
  const __attribute__((address_space(4))) NearCTile<T>* tile =
      (const __attribute__((address_space(4))) NearCTile<T>*)ws.items + ti;
  const uint32_t smask = tile->src_mask;
  const int ry = wave & 1, rz = wave >> 1;
  const bool has_row = (tile->row_mask >> wave) & 1u;
  const int nreal = tile->nreal, zero = tile->zero;
  const int nsc = (nreal + EPC - 1) / EPC;               // source copies, then kernel copies
  const cptr64 kp = (cptr64)tile->kptr;
  const gview<const T> Ft = gl((const T*)tile->fhat);
  // 16 bytes (2 FP32 or 1 FP64 frequencies) per lane; with FP32 lanes 0-31 copy the first entry
  // of a pair and lanes 32-63 the second
  const int sub = lane / LPE, lo = (lane % LPE) * (16 / (int)sizeof(T));
  // copy chunk c into buffer dst: copy m < nsc + 14 / EPC on wavefront m % WAVES
  auto issue = [&](cpx<T>* dst, int c) {
    for (int m = wave; m < nsc + kNearHalfK / EPC; m += WAVES) {
      gview<const T> src;
      int e0;
      if (m < nsc) {
        const int s0 = EPC * m < nreal ? tile->src[EPC * m] : zero;
        int sl = s0;
        if constexpr (EPC == 2) {
          const int s1 = 2 * m + 1 < nreal ? tile->src[2 * m + 1] : zero;
          sl = sub ? s1 : s0;
        }
        src = Ft + 2 * ((int64_t)sl * S + (int64_t)c * 64) + lo;
        e0 = EPC * m;
      } else {
        const int h = EPC * (m - nsc);
        gview<const T> kb = gl((const T*)kp[h]);
        if constexpr (EPC == 2) {
          const gview<const T> k1 = gl((const T*)kp[h + 1]);
          kb = sub ? k1 : kb;
        }
        src = kb + 2 * (int64_t)c * 64 + lo;
        e0 = KE + h;
      }
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                       (__attribute__((address_space(3))) void*)&dst[e0 * 64], 16, 0, 0);
    }
  };
  gmut<T> U = (gmut<T>)tile->uhat;
  // a tile without sources at x0 - 1 and x0 + 4 (a level no wider than its row, as on small
  // uniform layouts) skips the products with those positions: a sixth of the multiply-adds and
  // a third of the LDS reads
  const bool edges = tile->edges != 0;
  auto apply_e = [&](const cpx<T>* fb, int c, auto has_edges) {
    constexpr bool EDGES = decltype(has_edges)::value;
    cpx<T> kv[kNearHalfK];
#pragma unroll
    for (int h = 0; h < kNearHalfK; ++h) kv[h] = fb[(KE + h) * 64 + lane];
    cpx<T> acc[W];
#pragma unroll
    for (int q = 0; q < W; ++q) acc[q] = {T(0), T(0)};
#pragma unroll
    for (int pj = 0; pj < 9; ++pj) {
      const int dz = pj / 3 - 1, dy = pj % 3 - 1;
      const int q = (ry + 1 - dy) + 4 * (rz + 1 - dz);
      if (!((smask >> q) & 1u)) continue;
      cpx<T> fd[NS];
#pragma unroll
      for (int s2 = 0; s2 < NS; ++s2)
        if (EDGES || (s2 > 0 && s2 < NS - 1)) fd[s2] = fb[tile->loff[q * NS + s2] + lane];
#pragma unroll
      for (int dxi = 0; dxi < 3; ++dxi) {
        const int h = pj * 3 + dxi;
        const cpx<T> kk = h < kNearHalfK ? kv[h] : cpx<T>{kv[26 - h].x, -kv[26 - h].y};
#pragma unroll
        for (int x = 0; x < W; ++x) {                 // src x = x0 + x - dx
          const int e = x - dxi + 2;
          if (EDGES || (e > 0 && e < NS - 1)) cmac(acc[x], kk, fd[e]);
        }
      }
    }
    const int k = c * 64 + lane;
#pragma unroll
    for (int x = 0; x < W; ++x) {
      const int t = tile->tgt[wave][x];
      if (t >= 0) {
        U[2 * ((int64_t)t * S + k)] = acc[x].x;
        U[2 * ((int64_t)t * S + k) + 1] = acc[x].y;
      }
    }
  };
  // apply chunk c from buffer fb
  auto apply = [&](const cpx<T>* fb, int c) {
    if (!has_row) return;
    if (edges) apply_e(fb, c, std::true_type{});
    else apply_e(fb, c, std::false_type{});
  };
  if (wave == 0) {
    fa[NC * 64 + lane] = cpx<T>{T(0), T(0)};
    fz[NC * 64 + lane] = cpx<T>{T(0), T(0)};
  }
  issue(fa, c0);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  // chunks alternate between the buffers; after each chunk every wavefront waits for its copies
  // (and stores), and the barrier makes the copies visible and ends the reads of the buffer the
  // next copies go to
  for (int i = 0; i < nrun; i += 2) {
    if (i + 1 < nrun) issue(fz, c0 + i + 1);
    apply(fa, c0 + i);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (i + 1 >= nrun) break;
    if (i + 2 < nrun) issue(fa, c0 + i + 2);
    apply(fz, c0 + i + 1);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }
}

// Fused form: the base-level convolution of one tile for one group of (kx, ky) lines (one line
// of P = 64 frequencies kz for N_b = 16, two of 32 for N_b = 8: 64 values per column either
// way), from the line-major planes of the forward (x, y) pass to the line-major planes of the
// inverse one.  The z transforms are split as P = 8 Q (Cooley-Tukey, Q = P / 8) so that 8 or 16
// lanes share a column and each holds 4 to 8 values:
//   forward, zero-padded (z < P/2 = 4 Q nonzero): with z = Q n1 + n2 and kz = k1 + 8 k2,
//     Y[n2][k1] = W_P^{n2 k1} sum_{n1 < 4} x[Q n1 + n2] W_8^{n1 k1}   (lane n2: an 8-point DFT of 4 inputs)
//     X[k1 + 8 k2] = sum_{n2 < Q} Y[n2][k1] W_Q^{n2 k2}               (lane k1: a Q-point DFT)
//   inverse, cropped to z < P/2: with kz = Q k1 + k2 and z = n1 + 8 n2,
//     Z[k2][n1] = W_P^{-n1 k2} sum_{k1 < 8} X[Q k1 + k2] W_8^{-n1 k1}  (lane k2: an 8-point DFT)
//     x[n1 + 8 n2] = sum_{k2 < Q} Z[k2][n1] W_Q^{-n2 k2}, n2 < Q/2      (lane n1: a Q-point DFT)
// Each step of a transform writes back to the LDS positions it read (Y[n2][k1] at 8 n2 + k1,
// X[k1 + 8 k2] there too; Z[k2][n1] at Q n1 + k2), so no barrier separates its reads and writes.
// The 1 / P^3 of the inverse transform is left to the inverse (y, x) pass.
//
// Persistent workgroups: each takes the units (tile, line group) w, w + G, w + 2 G, ... of the
// launch (G workgroups, a multiple of 8, so that a workgroup keeps to the XCD of its units; the
// units of one line group lie on one XCD and share its source and kernel columns in L2).  Loads
// return in issue order, so each is issued where no earlier wait has to cover it: the source
// slots of the next unit after the forward step 1, its source columns (into registers) at the
// start of the MAC, its 14 kernel values after the MAC, while the inverse transforms run.  A
// wavefront owns RPW = 2 target rows (ry = 0, 1 at rz = its index) and walks the 4 x 3 source
// rows they draw from, each loaded once for both (one row per wavefront: more wavefronts, more
// LDS reads, slower); the LDS entries of those rows sit in two registers and are taken with
// readlane.  Every lane keeps its 8 twiddles W_P^{m k}, m = its position mod Q, for the whole
// launch: the forward step 1 (m = n2) and the inverse step 1 (m = k2) use the same ones.
template <typename T, int B2, int RZ, int NC, int RPW>
__global__ __launch_bounds__(128 * RZ / RPW) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 && B2 == 32 ? 3 : 1)))
void near_fused_kernel(SetTable sets, int64_t slot, int64_t units) {
  constexpr int P = 2 * B2, H = B2 + 1, PLANE = P * H, Q = P / 8;
  constexpr int LPW = 64 / P;                    // lines per unit
  constexpr int NGRP = PLANE / LPW;              // line groups
  constexpr int W = kTileW, NS = W + 2, NT = 2 * RZ * W, NTH = 128 * RZ / RPW;
  constexpr int IPT = (8 * NC + NTH - 1) / NTH;  // forward step 1 items per thread
  // LDS column layout.  FP32: value m of an entry's 64 at m + m / 8 (one pad per 8), entries 72
  // apart.  FP64: at m + m / 16, entries 68 apart, and the twiddles in an LDS table instead of
  // registers: 53 KB of LDS and at most 168 registers per lane, so three workgroups share a CU
  // (alone 71 -> 72.5 us on the 8^3 x 16^3 workload, in the solve 0.201-0.203 -> 0.197-0.198 ms:
  // the third workgroup takes up the CUs that the far field's kernels free)
  constexpr bool X64 = sizeof(T) == 8;
  constexpr int FS = X64 ? 68 : 72;
  auto at = [](int m) { return X64 ? m + (m >> 4) : m + (m >> 3); };
  static_assert(PLANE % LPW == 0 && NGRP % 8 == 0 && LPW * Q == 8 && NT <= NC && NT * 8 <= NTH, "column shape");
  __shared__ cpx<T> F[(NC + 1) * FS];            // source spectra (entry NC: zeros), then target spectra
  __shared__ cpx<T> TWL[X64 ? 64 : 1];           // FP64 twiddles W_P^{m k} at 8 k + m
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  // twiddles W_P^{m k}, k < 8, m = this thread's n2 (forward step 1) = k2 (inverse step 1)
  cpx<T> tw[X64 ? 1 : 8];
  if constexpr (X64) {
    if (tid < 64) {
      const int m = (tid & 7) % Q, k = tid >> 3;
      double sn, cs;
      sincospi(2.0 * ((m * k) % P) / P, &sn, &cs);
      TWL[tid] = cpx<T>{T(cs), T(-sn)};
    }
  } else {
    const int m = (tid & 7) % Q;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      double sn, cs;
      sincospi(2.0 * ((m * k) % P) / P, &sn, &cs);
      tw[k] = cpx<T>{T(cs), T(-sn)};
    }
  }
  auto twid = [&](int k) {
    if constexpr (X64) return TWL[8 * k + (tid & 7) % Q];
    else return tw[k];
  };
  if (tid < 64) F[NC * FS + at(tid)] = cpx<T>{T(0), T(0)};
  if constexpr (X64) __syncthreads();            // the twiddle table is read by every wavefront
  struct Unit {
    const __attribute__((address_space(4))) NearCTile<T>* tile;
    int line0;
  };
  auto unit_of = [&](int64_t u) {
    const WorkSet& ws = sets.s[find_set(sets, u)];
    const int64_t local = u - ws.wg_begin;       // wg_begin (first unit of the set) is a multiple of 8
    const int64_t jj = local >> 3;
    const int grp = (int)(jj / ws.count) * 8 + (int)(local & 7);
    Unit r;
    r.tile = (const __attribute__((address_space(4))) NearCTile<T>*)ws.items + jj % ws.count;
    r.line0 = grp * LPW;
    return r;
  };
  // forward step 1 inputs of a unit: item i = 8 e + (ls, n2) loads x[Q n1 + n2], n1 < 4, of line
  // line0 + ls of staged entry e.  The slots of the entries are read first (fetch_slots), the
  // values later (fetch_values), so that the value loads go out without waiting.  Every load is
  // issued unconditionally (items past the staged entries read the all-zero slot, which src[]
  // holds past nreal), so that the waits for the kernel values, issued before them, are exact.
  T xr[IPT][4], xi[IPT][4];
  int slots[IPT];
  int nnext = 0;
  auto fetch_slots = [&](const Unit& un) {
    nnext = un.tile->nreal;
#pragma unroll
    for (int j = 0; j < IPT; ++j) slots[j] = un.tile->src[min((tid + j * NTH) >> 3, NC - 1)];
  };
  auto fetch_values = [&](const Unit& un) {
    const gview<const T> Fp = gl((const T*)un.tile->fhat);
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
      const int r = (tid + j * NTH) & 7, ls = r / Q, n2 = r % Q;
      const int64_t col = 2 * ((int64_t)slots[j] * slot + (int64_t)(un.line0 + ls) * B2);
#pragma unroll
      for (int n1 = 0; n1 < 4; ++n1) {
        xr[j][n1] = Fp[col + 2 * (Q * n1 + n2)];
        xi[j][n1] = Fp[col + 2 * (Q * n1 + n2) + 1];
      }
    }
  };
  // the 14 kernel values of a lane's (line, kz) of a unit (L2, or HBM on the first tile of a
  // line group); requested a unit ahead, while the previous unit's inverse transforms run
  cpx<T> kv[kNearHalfK];
  auto fetch_kernels = [&](const Unit& un) {
    const gview<const T> Kc = gl((const T*)un.tile->ktr);
#pragma unroll
    for (int h = 0; h < kNearHalfK; ++h) {
      const int64_t o = 2 * (((int64_t)h * PLANE + un.line0) * P + lane);
      kv[h] = cpx<T>{Kc[o], Kc[o + 1]};
    }
  };
  // With one line per unit, the 8 lanes of a column (forward steps) and the entries of a target
  // (its accumulator store and the inverse steps) belong to one wavefront, so between those
  // steps, and between a unit's inverse steps and the next unit's forward step 1 (which writes
  // only the wavefront's own target entries and source entries that no other wavefront reads
  // after the MAC's barrier), LDS needs ordering within the wavefront only; LDS operations of a
  // wavefront complete in order.  Only the barriers around the MAC (all wavefronts read every
  // source entry, then the targets overwrite them) order the whole workgroup.
  auto wave_sync = [&]() {
    if constexpr (LPW == 1) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
      __syncthreads();
    }
  };
  int64_t u = blockIdx.x;
  if (u >= units) return;
  Unit cur = unit_of(u);
  fetch_slots(cur);
  fetch_values(cur);
  fetch_kernels(cur);
  for (; u < units; u += gridDim.x) {
    const auto* tile = cur.tile;
    const int line0 = cur.line0;
    const int nreal = nnext;
    int tg[LPW];                                 // the inverse step 2's targets
#pragma unroll
    for (int j = 0; j < LPW; ++j) {
      const int jt = min((tid + j * NTH) / (8 * LPW), NT - 1);
      tg[j] = tile->tgt[jt / W][jt % W];
    }
    // the LDS entries of the wavefront's source rows (rows 4 rz .. 4 rz + 11, NS each) in two
    // registers, lane l holding entry 24 rz + l and 24 rz + 64 + l: the MAC takes them with
    // readlane at compile-time lanes instead of scalar loads (which would share the LDS wait
    // counter and serialise the rows)
    const int lbase = 4 * NS * ((wave * RPW) >> 1);
    const uint32_t lv0 = tile->loff[min(lbase + lane, kTileSrcRowsMax * NS - 1)];
    const uint32_t lv1 = tile->loff[min(lbase + 64 + lane, kTileSrcRowsMax * NS - 1)];
    // the next unit (the last one refetches its own inputs, unused)
    if (u + gridDim.x < units) cur = unit_of(u + gridDim.x);
    wave_sync();                                 // this wavefront's reads of its entries are done
    // 1. forward step 1 from the prefetched inputs
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
      const int i = tid + j * NTH;
      if (i < 8 * nreal) {
        const int e = i >> 3, r = i & 7, ls = r / Q, n2 = r % Q;
        T yr[8], yi[8];
        fwd_padded<4>(xr[j], xi[j], yr, yi);
#pragma unroll
        for (int k1 = 0; k1 < 8; ++k1) {
          const cpx<T> w = twid(k1);               // W_P^{n2 k1}
          F[e * FS + at(ls * P + n2 * 8 + k1)] =
              k1 ? cpx<T>{yr[k1] * w.x - yi[k1] * w.y, yr[k1] * w.y + yi[k1] * w.x} : cpx<T>{yr[0], yi[0]};
        }
      }
    }
    fetch_slots(cur);
    wave_sync();
    // 2. forward step 2 in place: item (entry, line, k1)
    for (int i = tid; i < 8 * LPW * nreal; i += NTH) {
      const int e = i / (8 * LPW), r = i % (8 * LPW), ls = r >> 3, k1 = r & 7;
      T vr[Q], vi[Q];
#pragma unroll
      for (int n2 = 0; n2 < Q; ++n2) {
        const cpx<T> v = F[e * FS + at(ls * P + n2 * 8 + k1)];
        vr[n2] = v.x;
        vi[n2] = v.y;
      }
      fft_inreg<Q, -1>(vr, vi);
#pragma unroll
      for (int k2 = 0; k2 < Q; ++k2) F[e * FS + at(ls * P + k1 + 8 * k2)] = cpx<T>{vr[k2], vi[k2]};
    }
    __syncthreads();
    // 3. MAC: wavefront = RPW target rows, lane = (line, kz), the kernel values requested during
    // the previous unit; the next unit's inputs are requested first.
    cpx<T> acc[RPW][W];
    {
      fetch_values(cur);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int j = 0; j < RPW; ++j)
#pragma unroll
        for (int x = 0; x < W; ++x) acc[j][x] = {T(0), T(0)};
      const uint32_t smask = tile->src_mask;
      const int r0 = wave * RPW;                 // the wavefront's rows r0 .. r0 + RPW - 1
      const int ry0 = r0 & 1, rz = r0 >> 1;      // (RPW = 2: both rows at rz)
      auto mac = [&](auto has_edges) {
        constexpr bool EDGES = decltype(has_edges)::value;
#pragma unroll
        for (int qzi = 0; qzi < 3; ++qzi) {
#pragma unroll
          for (int qyi = 0; qyi < RPW + 2; ++qyi) {
            const int q = ry0 + qyi + 4 * (rz + qzi);   // source row (y0 - 1 + qy, z0 - 1 + rz + qzi)
            if (!((smask >> q) & 1u)) continue;
            cpx<T> fd[NS];
#pragma unroll
            for (int s2 = 0; s2 < NS; ++s2)
              if (EDGES || (s2 > 0 && s2 < NS - 1)) {
                const int li = (ry0 + qyi + 4 * qzi) * NS + s2;   // q NS + s2 - lbase
                const uint32_t off = __builtin_amdgcn_readlane(li < 64 ? lv0 : lv1, li & 63);
                fd[s2] = F[(off >> 6) * FS + at(lane)];
              }
#pragma unroll
            for (int j = 0; j < RPW; ++j) {
              const int dyi = j + 2 - qyi;         // dy + 1 of target row ry0 + j
              if (dyi < 0 || dyi > 2) continue;
              const int pj = 3 * (2 - qzi) + dyi;  // 3 (dz + 1) + dy + 1
#pragma unroll
              for (int dxi = 0; dxi < 3; ++dxi) {
                const int h = pj * 3 + dxi;
                const cpx<T> kk = h < kNearHalfK ? kv[h] : cpx<T>{kv[26 - h].x, -kv[26 - h].y};
#pragma unroll
                for (int x = 0; x < W; ++x) {     // src x = x0 + x - dx
                  const int e = x - dxi + 2;
                  if (EDGES || (e > 0 && e < NS - 1)) cmac(acc[j][x], kk, fd[e]);
                }
              }
            }
          }
        }
      };
      if ((tile->row_mask >> r0) & ((1u << RPW) - 1)) {
        if (tile->edges) mac(std::true_type{});
        else mac(std::false_type{});
      }
    }
    __syncthreads();                             // every source spectrum is consumed
#pragma unroll
    for (int j = 0; j < RPW; ++j)
#pragma unroll
      for (int x = 0; x < W; ++x) F[((wave * RPW + j) * W + x) * FS + at(lane)] = acc[j][x];
    wave_sync();
    // 4. inverse step 1 in place: item (target, line, k2) = this thread; Z[k2][n1] goes to the
    // position Q n1 + k2 of X[Q n1 + k2]
    __builtin_amdgcn_sched_barrier(0);
    fetch_kernels(cur);                          // the next unit's (kv is free after the MAC)
    __builtin_amdgcn_sched_barrier(0);
    if (tid < 8 * NT) {
      const int jt = tid >> 3, r = tid & 7, ls = r / Q, k2 = r % Q;
      T zr[8], zi[8];
#pragma unroll
      for (int k1 = 0; k1 < 8; ++k1) {
        const cpx<T> v = F[jt * FS + at(ls * P + Q * k1 + k2)];
        zr[k1] = v.x;
        zi[k1] = v.y;
      }
      fft_inreg<8, +1>(zr, zi);
#pragma unroll
      for (int n1 = 0; n1 < 8; ++n1) {
        const cpx<T> w = twid(n1);                 // W_P^{n1 k2}, conjugated
        F[jt * FS + at(ls * P + Q * n1 + k2)] =
            n1 ? cpx<T>{zr[n1] * w.x + zi[n1] * w.y, zi[n1] * w.x - zr[n1] * w.y} : cpx<T>{zr[0], zi[0]};
      }
    }
    wave_sync();
    // 5. inverse step 2: item (target, line, n1); store z = n1 + 8 n2 < B2
    {
      gmut<T> U = (gmut<T>)tile->uhat;
#pragma unroll
      for (int j = 0; j < LPW; ++j) {
        const int i = tid + j * NTH;
        const int jt = i / (8 * LPW), r = i % (8 * LPW), ls = r >> 3, n1 = r & 7;
        const int t = tg[j];
        if (jt >= NT || t < 0) continue;
        T vr[Q], vi[Q], zr[Q / 2], zi[Q / 2];
#pragma unroll
        for (int k2 = 0; k2 < Q; ++k2) {
          const cpx<T> v = F[jt * FS + at(ls * P + Q * n1 + k2)];
          vr[k2] = v.x;
          vi[k2] = v.y;
        }
        inv_cropped<Q / 2>(vr, vi, zr, zi);
        const int64_t col = 2 * ((int64_t)t * slot + (int64_t)(line0 + ls) * B2);
#pragma unroll
        for (int n2 = 0; n2 < Q / 2; ++n2) {
          U[col + 2 * (n1 + 8 * n2)] = zr[n2];
          U[col + 2 * (n1 + 8 * n2) + 1] = zi[n2];
        }
      }
    }
  }
}

template <typename T, int B2, int RZ>
hipError_t launch_fused_rz(SetTable& t, hipStream_t st) {
  constexpr int P = 2 * B2, PLANE = P * (B2 + 1), NGRP = PLANE / (64 / P);
  constexpr int NC = near_ctile_cap(RZ == 2 ? kNearFused + 2 : kNearFused + 4);
  constexpr int RPW = 2, NTH = 128 * RZ / RPW;
  const int64_t S = (int64_t)P * PLANE;               // complex entries per super-block slot
  int64_t units = 0;
  for (int i = 0; i < t.n; ++i) {
    t.s[i].wg_begin = units;
    units += (int64_t)t.s[i].count * NGRP;
  }
  if (units == 0) return hipSuccess;
  // persistent workgroups (a multiple of 8), each walking its units
  static int resident = 0;
  if (resident == 0) {
    int per_cu = 0, dev = 0, cus = 0;
    LGF_HIP_CHECK(hipGetDevice(&dev));
    LGF_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    LGF_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, near_fused_kernel<T, B2, RZ, NC, RPW>,
                                                               NTH, 0));
    resident = std::max(8, (per_cu * cus) / 8 * 8);
  }
  // two rounds of the resident count: beside the far field's kernels (which hold CUs when this
  // launch starts) the second round's workgroups start where CUs free up first, so the units
  // follow the free CUs instead of waiting on workgroups that are not resident yet; alone, two
  // full rounds cost nothing over one (FP64 solve of the 8^3 x 16^3 workload 0.214 -> 0.207 ms,
  // kernel alone 70.5 us either way; three rounds 71.2 us, four 74.5 us)
  const int64_t wg = std::min<int64_t>(2 * (int64_t)resident, (units + 7) / 8 * 8);
  near_fused_kernel<T, B2, RZ, NC, RPW><<<(unsigned)wg, NTH, 0, st>>>(t, S, units);
  return hipGetLastError();
}

template <typename T, int B2>
hipError_t launch_fused_b2(SetTable& t, hipStream_t st, int mode) {
  if (mode == kNearFused + 2) return launch_fused_rz<T, B2, 2>(t, st);
  return launch_fused_rz<T, B2, 4>(t, st);
}

}  // namespace

// mode: targets per row W (2, 4 or 8) with NearRow items, kNearTiled + 4 / + 6 with NearTile items
// of 2 x 2 / 2 x 4 rows;
// chosen by the planner.  All rows of a work set share one kernel table (the wavefronts of a
// workgroup stage the kernels for all its rows).
template <typename T> hipError_t launch_near_mac(int nb, SetTable& t, hipStream_t st, int mode) {
  if (near_fused(mode)) {
    if (nb == 16) return launch_fused_b2<T, 32>(t, st, mode);
    if (nb == 8) return launch_fused_b2<T, 16>(t, st, mode);
    return hipErrorInvalidValue;
  }
  const int B2 = 2 * nb, P = 2 * B2;
  const int S = P * P * (B2 + 1);
  if (S % 64) return hipErrorInvalidValue;
  const int chunks8 = (S / 64 + 7) / 8;
  const bool tiled = mode > kNearTiled;
  const bool piped = near_piped(mode);
  // pipelined form: runs of 2 to 8 chunks per workgroup, longer where the launch has work for
  // more than about 2048 workgroups (small levels need the workgroups, large ones the pipeline)
  int RUN = kNearRunMin;
  if (piped) {
    int64_t tiles = 0;
    for (int i = 0; i < t.n; ++i) tiles += t.s[i].count;
    while (RUN < kNearRunMax && tiles * (S / 64) / (2 * RUN) >= 2048) RUN *= 2;
  }
  const int runs8 = (S / 64 / RUN + 7) / 8 + 1;     // runs of chunks per XCD (covering)
  int64_t wg = 0;
  for (int i = 0; i < t.n; ++i) {
    t.s[i].wg_begin = wg;
    wg += piped ? (int64_t)t.s[i].count * runs8 * 8
                : (int64_t)(tiled ? t.s[i].count : (t.s[i].count + 3) / 4) * chunks8 * 8;
  }
  if (wg == 0) return hipSuccess;
  if (mode == 2) near_mac_kernel<T, 2><<<(unsigned)wg, 256, 0, st>>>(t, S);
  else if (mode == 4) near_mac_kernel<T, 4><<<(unsigned)wg, 256, 0, st>>>(t, S);
  else if (mode == 8) near_mac_kernel<T, 8><<<(unsigned)wg, 256, 0, st>>>(t, S);
  else if (mode == kNearTiled + 4) near_tile_kernel<T, kTileW, 2><<<(unsigned)wg, 256, 0, st>>>(t, S);
  else if (mode == kNearTiled + 6) near_tile_kernel<T, kTileW, 4><<<(unsigned)wg, 512, 0, st>>>(t, S);
  else if (piped) {
    if (mode == kNearTiled + 5) near_pipe_kernel<T, 2, near_ctile_cap(kNearTiled + 5)><<<(unsigned)wg, 256, 0, st>>>(t, S, RUN);
    else near_pipe_kernel<T, 4, near_ctile_cap(kNearTiled + 7)><<<(unsigned)wg, 512, 0, st>>>(t, S, RUN);
  }
  else return hipErrorInvalidValue;
  return hipGetLastError();
}


template hipError_t launch_near_mac<float>(int, SetTable&, hipStream_t, int);
template hipError_t launch_near_mac<double>(int, SetTable&, hipStream_t, int);

}  // namespace lgf
