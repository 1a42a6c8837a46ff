// Spectral multiply-accumulate of the level interaction (Sec. 2.1, Algorithm 1 step 2):
//   U_t[k] = sum over the interaction list of t of K_{s, t-src}[k] * F_src[k]
// for every frequency k of the half spectrum.  The list of a target follows from its parity
// (Fig. fmm_regions): its sources are the children of its parent's neighbours, i.e. the offsets
// d = t - src with c_i - 3 <= d_i <= c_i + 2 (c = parity of t); on coarse levels the near region
// |d|_inf <= 1 is excluded, on the base level it is included.
//
// Work unit: a tile of 2x2 sibling target rows (8 targets along x each) and 64 consecutive
// frequencies (one per lane).  Siblings share their parent's neighbours, so the four rows draw
// from the same 36 source rows.  A wavefront accumulates ROWS of the tile's rows (1, 2 or 4):
// for each source row it holds the 14 source spectra of the x window in registers and reuses
// them against the 7 kernel offsets along x and its rows.  The next source row's spectra (and,
// without LDS staging, its kernel spectra) are loaded before the current row's arithmetic, so a
// single wait per source row covers the memory latency.  In FP32 the kernel spectra of the
// level are staged in LDS for the workgroup's 64 frequencies; only offsets d >= 0
// (lexicographically) are stored: the kernel is real and even in every coordinate, so
// K_{-d}[k] = conj(K_d[k]).  All control flow is uniform per wavefront.
#include <cstdlib>
#include <cstring>

#include "kernels.hpp"

namespace lgf {

namespace {

constexpr int kHalfK = 172;      // offsets with (dz, dy, dx) >= 0 lexicographically: index <= 171

template <typename T> using gptr = const __attribute__((address_space(1))) T*;
template <typename T> using gmut = __attribute__((address_space(1))) T*;
using cptr64 = const __attribute__((address_space(4))) uint64_t*;   // scalar-loadable table

template <typename T> __device__ __forceinline__ cpx<T> gload(gptr<T> base, int64_t i) {
  return {base[2 * i], base[2 * i + 1]};
}

// absent sources point at the arena's all-zero spectrum, so every load is unconditional
template <typename T>
__device__ __forceinline__ void load_src(cpx<T> (&fs)[kMacSlots], const int32_t* __restrict__ sr,
                                         gptr<T> F, int S, int k) {
#pragma unroll
  for (int s = 0; s < kMacSlots; ++s) fs[s] = gload<T>(F, (int64_t)sr[s] * S + k);
}

__device__ __forceinline__ int kindex(int r, int jz, int jy, int dxi) {
  const int ry = r & 1, rz = r >> 1;
  return (rz + 5 - jz) * 49 + (ry + 5 - jy) * 7 + dxi;   // (dz+3)*49 + (dy+3)*7 + dx+3
}

template <typename T, int ROWS>
__device__ __forceinline__ void load_k(cpx<T> (&ks)[ROWS][7], cptr64 kp, int r0, int jz, int jy, int k) {
#pragma unroll
  for (int q = 0; q < ROWS; ++q)
#pragma unroll
    for (int dxi = 0; dxi < 7; ++dxi) {
      const uint64_t p = kp[kindex(r0 + q, jz, jy, dxi)];
      ks[q][dxi] = gload<T>((gptr<T>)p, k);
    }
}

// accumulate one source row (jz, jy) into target row r with kernel values kv(dxi)
template <typename T, typename KF>
__device__ __forceinline__ void mac_row(cpx<T> (&acc)[kMacL], const cpx<T> (&fs)[kMacSlots], int r, int jz,
                                        int jy, bool base, KF&& kv) {
  const int ry = r & 1, rz = r >> 1;
  const int dz = rz + 2 - jz, dy = ry + 2 - jy;
  const bool near_zy = dz >= -1 && dz <= 1 && dy >= -1 && dy <= 1;
#pragma unroll
  for (int dxi = 0; dxi < 7; ++dxi) {
    const int dx = dxi - 3;
    if (!base && near_zy && dx >= -1 && dx <= 1) continue;
    const cpx<T> kk = kv(dxi);
#pragma unroll
    for (int i = 0; i < kMacL; ++i) {
      const int c = i & 1;
      if (dx < c - 3 || dx > c + 2) continue;
      cmac(acc[i], kk, fs[i - dx + 3]);
    }
  }
}

// SPLIT = 6: the six waves of a workgroup share one (tile, row group) and take one source-row
// plane jz each; their partial sums are added in a fixed order through LDS (for small levels).
template <typename T, int WAVES, int ROWS, bool KLDS, int SPLIT>
__global__ __launch_bounds__(64 * WAVES) void mac_tile_kernel(SetTable sets, int S) {
  __shared__ cpx<T> klds[KLDS ? kHalfK * 64 : 1];
  __shared__ cpx<T> red[SPLIT > 1 ? (SPLIT - 1) * ROWS * kMacL * 64 : 1];
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

  cpx<T> acc[ROWS][kMacL];
#pragma unroll
  for (int q = 0; q < ROWS; ++q)
#pragma unroll
    for (int i = 0; i < kMacL; ++i) acc[q][i] = {T(0), T(0)};

  if (todo) {
    int pj = __builtin_ctzll(todo);
    todo &= todo - 1;
    cpx<T> fs[kMacSlots];
    cpx<T> ks[KLDS ? 1 : ROWS][7];
    load_src<T>(fs, tile->src[pj], F, S, k);
    if constexpr (!KLDS) load_k<T, ROWS>(ks, kp, r0, pj / 6, pj % 6, k);
    for (;;) {
      const int pn = todo ? __builtin_ctzll(todo) : -1;
      cpx<T> fn[kMacSlots];
      cpx<T> kn[KLDS ? 1 : ROWS][7];
      if (pn >= 0) {
        todo &= todo - 1;
        load_src<T>(fn, tile->src[pn], F, S, k);
        if constexpr (!KLDS) load_k<T, ROWS>(kn, kp, r0, pn / 6, pn % 6, k);
      }
      const int jz = pj / 6, jy = pj % 6;
#pragma unroll
      for (int q = 0; q < ROWS; ++q) {
        if (!((mymask >> q) & 1)) continue;
        const int r = r0 + q;
        if constexpr (KLDS) {
          mac_row<T>(acc[q], fs, r, jz, jy, base, [&](int dxi) {
            const int idx = kindex(r, jz, jy, dxi);
            const bool mirror = idx >= kHalfK;
            cpx<T> kv = klds[(mirror ? 342 - idx : idx) * 64 + lane];
            if (mirror) kv.y = -kv.y;
            return kv;
          });
        } else {
          mac_row<T>(acc[q], fs, r, jz, jy, base, [&](int dxi) { return ks[q][dxi]; });
        }
      }
      if (pn < 0) break;
#pragma unroll
      for (int s = 0; s < kMacSlots; ++s) fs[s] = fn[s];
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
        for (int i = 0; i < kMacL; ++i) red[(((part - 1) * ROWS + q) * kMacL + i) * 64 + lane] = acc[q][i];
    }
    __syncthreads();
    if (part > 0) return;
    for (int p = 1; p < SPLIT; ++p)
#pragma unroll
      for (int q = 0; q < ROWS; ++q)
#pragma unroll
        for (int i = 0; i < kMacL; ++i) {
          const cpx<T> v = red[(((p - 1) * ROWS + q) * kMacL + i) * 64 + lane];
          acc[q][i].x += v.x;
          acc[q][i].y += v.y;
        }
  }
  gmut<T> U = (gmut<T>)tile->uhat;
#pragma unroll
  for (int q = 0; q < ROWS; ++q)
#pragma unroll
    for (int i = 0; i < kMacL; ++i) {
      const int t = tile->tgt[r0 + q][i];
      if (t >= 0) {
        U[2 * ((int64_t)t * S + k)] = acc[q][i].x;
        U[2 * ((int64_t)t * S + k) + 1] = acc[q][i].y;
      }
    }
}

template <typename T, int WAVES, int ROWS, bool KLDS, int SPLIT = 1>
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
  mac_tile_kernel<T, WAVES, ROWS, KLDS, SPLIT><<<(unsigned)wg, 64 * WAVES, 0, st>>>(t, S);
  return hipGetLastError();
}

}  // namespace

// Launch shape (mode): 1 row, 2 pair, 4 tile = rows per wavefront; 6 split = FP64 source rows
// over 6 wavefronts; 0 = default (one row per wavefront; FP32 with the kernel spectra in LDS and
// 16 wavefronts per workgroup, FP64 with the kernel spectra prefetched from memory).  The plan's
// autotuner picks the mode per step; LGF_MAC_MODE = row | pair | tile | split overrides it.
int mac_mode_override() {
  static const int m = [] {
    const char* e = std::getenv("LGF_MAC_MODE");
    if (!e) return 0;
    if (!std::strcmp(e, "row")) return 1;
    if (!std::strcmp(e, "pair")) return 2;
    if (!std::strcmp(e, "tile")) return 4;
    if (!std::strcmp(e, "split")) return 6;
    return 0;
  }();
  return m;
}

template <typename T> hipError_t launch_mac(int nb, SetTable& t, hipStream_t st, int mode) {
  const int P = 2 * nb;
  const int S = P * P * (nb + 1);          // multiple of 64 for nb in {8, 16}
  if (S % 64) return hipErrorInvalidValue;
  if (const int o = mac_mode_override()) mode = o;
  if constexpr (sizeof(T) == 4) {
    if (mode == 4) return launch_tiles<T, 16, 4, true>(S, t, st);
    if (mode == 2) return launch_tiles<T, 16, 2, true>(S, t, st);
    return launch_tiles<T, 16, 1, true>(S, t, st);
  } else {
    if (mode == 2) return launch_tiles<T, 4, 2, false>(S, t, st);
    if (mode == 6) return launch_tiles<T, 6, 1, false, 6>(S, t, st);
    return launch_tiles<T, 4, 1, false>(S, t, st);
  }
}

template hipError_t launch_mac<float>(int, SetTable&, hipStream_t, int);
template hipError_t launch_mac<double>(int, SetTable&, hipStream_t, int);

}  // namespace lgf
