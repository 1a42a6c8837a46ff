// Spectral multiply-accumulate of the level interaction (Sec. 2.1, Algorithm 1 step 2):
//   U_t[k] = sum over the interaction list of t of K_{s, t-src}[k] * F_src[k]
// for every frequency k of the half spectrum.  The list of a target is read from its parity
// (Fig. fmm_regions): the sources are the children of the neighbours of t's parent, i.e. the
// offsets d = t - src with c_i - 3 <= d_i <= c_i + 2 (c = parity of t); at coarse levels the
// near region |d|_inf <= 1 is excluded, at the base level it is included.
//
// A row is a run of up to 8 targets along x starting at an even x.  One wavefront owns one row
// and 64 consecutive frequencies; for each (dy, dz) it loads the 14 source spectra of the row's
// x window into registers once and reuses each against the 7 kernel spectra of that (dy, dz),
// so every loaded complex number feeds up to 6 targets.  Control flow is uniform per wave.
#include "kernels.hpp"

namespace lgf {

namespace {

constexpr int kMacThreads = 256;

template <typename T>
__global__ __launch_bounds__(kMacThreads) void mac_kernel(SetTable sets, int S) {
  const int set = find_set(sets, blockIdx.x);
  const WorkSet& ws = sets.s[set];
  const int64_t local = blockIdx.x - ws.wg_begin;
  const int nrows = ws.count;
  const int row_i = (int)(local % nrows);
  const int chunk = (int)(local / nrows);
  const MacRow<T>* row = (const MacRow<T>*)ws.items + row_i;
  const int k = chunk * kMacThreads + threadIdx.x;
  if (k >= S) return;

  const int flags = row->flags;
  const bool base = flags & 1;
  const int cy = (flags >> 1) & 1, cz = (flags >> 2) & 1;
  const uint64_t pmask = row->pair_mask;
  const cpx<T>* __restrict__ F = row->fhat;
  const cpx<T>* const* kptr = row->kptr;

  cpx<T> acc[kMacL];
#pragma unroll
  for (int i = 0; i < kMacL; ++i) acc[i] = {T(0), T(0)};

  for (int jz = 0; jz < 6; ++jz) {
    const int dz = cz - 3 + jz;
    for (int jy = 0; jy < 6; ++jy) {
      const int pj = jz * 6 + jy;
      if (!((pmask >> pj) & 1)) continue;
      const int dy = cy - 3 + jy;
      const int32_t* sr = row->src[pj];
      cpx<T> fs[kMacSlots];
#pragma unroll
      for (int s = 0; s < kMacSlots; ++s) {
        const int id = sr[s];
        fs[s] = id >= 0 ? F[(int64_t)id * S + k] : cpx<T>{T(0), T(0)};
      }
      const bool near_zy = dz >= -1 && dz <= 1 && dy >= -1 && dy <= 1;
      const cpx<T>* const* kp = kptr + (dz + 3) * 49 + (dy + 3) * 7;
#pragma unroll
      for (int dxi = 0; dxi < 7; ++dxi) {
        const int dx = dxi - 3;
        if (!base && near_zy && dx >= -1 && dx <= 1) continue;
        const cpx<T> kv = kp[dxi][k];
#pragma unroll
        for (int i = 0; i < kMacL; ++i) {
          const int c = i & 1;
          if (dx < c - 3 || dx > c + 2) continue;
          cmac(acc[i], kv, fs[i - dx + 3]);
        }
      }
    }
  }
  cpx<T>* U = row->uhat;
#pragma unroll
  for (int i = 0; i < kMacL; ++i) {
    const int t = row->tgt[i];
    if (t >= 0) U[(int64_t)t * S + k] = acc[i];
  }
}

}  // namespace

template <typename T> hipError_t launch_mac(int nb, SetTable& t, hipStream_t st) {
  const int P = 2 * nb;
  const int S = P * P * (nb + 1);
  const int chunks = (S + kMacThreads - 1) / kMacThreads;
  const int64_t wg = assign_wg(t, chunks);
  if (wg == 0) return hipSuccess;
  mac_kernel<T><<<(unsigned)wg, kMacThreads, 0, st>>>(t, S);
  return hipGetLastError();
}

template hipError_t launch_mac<float>(int, SetTable&, hipStream_t);
template hipError_t launch_mac<double>(int, SetTable&, hipStream_t);

}  // namespace lgf
