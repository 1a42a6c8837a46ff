// Zero-padded FFTs of base-level super-blocks.
//
// On the base octree level every target's interaction region (its near field N(B) plus its
// influence list I(B), Sec. 2.1) is exactly the set of children of its parent's 27 neighbours.
// The base-level interaction of all 8 children of a parent is therefore one block convolution of
// the parent-sized super-block (B2 = 2 N_b cells per side, zero-padded to P = 2 B2) with its 27
// neighbouring super-blocks, against the base-lattice kernel.  These kernels transform a
// super-block assembled from (up to) eight child blocks, and scatter the inverse transform's
// cropped output back to the children.
//
// Each direction takes two passes through a global intermediate plane stack
// T[z][ky][kx] (z < B2, ky < P, kx <= B2): the (x, y) pass transforms one z-plane per lane group,
// the z pass one (kx, ky) line per lane.  Every length-P line has only its first B2 entries
// nonzero (forward) or needed (inverse), so each is two length-B2 transforms.
#include "kernels.hpp"

namespace lgf {

namespace {

template <int B2> struct SupShape {
  static constexpr int P = 2 * B2;
  static constexpr int H = B2 + 1;               // kx in [0, B2]
  static constexpr int NB = B2 / 2;              // child block side
  static constexpr int PLANE = P * H;            // complex entries per intermediate plane
  static constexpr int S = P * P * H;
};

// 16-byte vectors of the child element type (rows are loaded whole, not element by element)
template <typename TC> struct Row16;
template <> struct Row16<float> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct Row16<double> { typedef double type __attribute__((ext_vector_type(2))); };

// row y of plane z of the assembled super-block: x < NB from the octant with cx = 0, the rest
// from cx = 1 (absent children read as zeros)
template <int NB, typename T, typename TC>
__device__ __forceinline__ void load_row(const SuperFwdItem<T>& it, const double* in, int y, int z,
                                         T (&xr)[2 * NB]) {
  using V = typename Row16<TC>::type;
  constexpr int E = 16 / sizeof(TC), NV = NB / E;
  const int oc0 = 2 * (y >= NB) + 4 * (z >= NB);
  const int off = ((z & (NB - 1)) * NB + (y & (NB - 1))) * NB;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const TC* c = child_ptr<TC>((const TC*)it.child[oc0 + h], it.child_in[oc0 + h], in);
    if (c) {
      const gview<const V> row = (gview<const V>)gl(c + off);
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        const V v = row[q];
#pragma unroll
        for (int e = 0; e < E; ++e) xr[h * NB + q * E + e] = T(v[e]);
      }
    } else {
#pragma unroll
      for (int x = 0; x < NB; ++x) xr[h * NB + x] = T(0);
    }
  }
}

// (item, z-plane) of a workgroup.  Plane-major (LM = 0): consecutive workgroups take consecutive
// planes.  Line-major (LM = 1): every plane of an item runs on one XCD (workgroup w goes to XCD
// w mod 8; set starts are multiples of 8), so the planes' scattered 8- or 16-byte pieces of
// each line meet in that XCD's L2 and leave it as whole lines.
template <int B2, bool LM>
__device__ __forceinline__ bool plane_of(const WorkSet& ws, int64_t local, int64_t* item, int* z) {
  if constexpr (!LM) {
    *item = local / B2;
    *z = (int)(local % B2);
    return true;
  }
  const int64_t r = local >> 3;
  *z = (int)(r % B2);
  *item = (r / B2) * 8 + (local & 7);
  return *item < ws.count;
}

// forward (x, y) pass: one workgroup per (super-block, z-plane); lanes own x-lines, then y-lines
// T: transform and spectrum type, TC: element type of the child blocks.  LM = 0: plane z goes to
// the plane stack T[z][line]; LM = 1: to the line-major planes T[line][z] (line = ky H + kx).
template <int B2, typename T, typename TC, bool LM>
__global__ __launch_bounds__(64) void sup_fwd_xy(SetTable sets) {
  using Sh = SupShape<B2>;
  constexpr int P = Sh::P, H = Sh::H, NB = Sh::NB;
  __shared__ cpx<T> pl[B2 * H];                 // [y][kx] after the x pass
  const int set = find_set(sets, blockIdx.x);
  const WorkSet& ws = sets.s[set];
  const int64_t local = blockIdx.x - ws.wg_begin;
  int64_t item;
  int z;
  if (!plane_of<B2, LM>(ws, local, &item, &z)) return;
  const SuperFwdItem<T>& it = ((const SuperFwdItem<T>*)ws.items)[item];
  const int tid = threadIdx.x;
  for (int y = tid; y < B2; y += 64) {
    T xr[B2], xi[B2], Xr[P], Xi[P];
    load_row<NB, T, TC>(it, ws.in, y, z, xr);
#pragma unroll
    for (int x = 0; x < B2; ++x) xi[x] = T(0);
    fwd_padded<B2>(xr, xi, Xr, Xi);
#pragma unroll
    for (int k = 0; k < H; ++k) pl[y * H + k] = {Xr[k], Xi[k]};
  }
  __syncthreads();
  cpx<T>* const out = LM ? it.tmp : it.tmp + (int64_t)z * Sh::PLANE;
  for (int kx = tid; kx < H; kx += 64) {
    T yr[B2], yi[B2], Yr[P], Yi[P];
#pragma unroll
    for (int y = 0; y < B2; ++y) { yr[y] = pl[y * H + kx].x; yi[y] = pl[y * H + kx].y; }
    fwd_padded<B2>(yr, yi, Yr, Yi);
#pragma unroll
    for (int ky = 0; ky < P; ++ky) {
      if constexpr (LM) gst(out, (int64_t)(ky * H + kx) * B2 + z, cpx<T>{Yr[ky], Yi[ky]});
      else gst(out, ky * H + kx, cpx<T>{Yr[ky], Yi[ky]});
    }
  }
}

// forward z pass: one lane per (kx, ky) line
template <int B2, typename T>
__global__ __launch_bounds__(256) void sup_fwd_z(SetTable sets) {
  using Sh = SupShape<B2>;
  constexpr int P = Sh::P, B = B2;
  constexpr int LINES = Sh::PLANE;
  constexpr int WG_PER_ITEM = (LINES + 255) / 256;
  const int set = find_set(sets, blockIdx.x);
  const WorkSet& ws = sets.s[set];
  const int64_t local = blockIdx.x - ws.wg_begin;
  const SuperFwdItem<T>& it = ((const SuperFwdItem<T>*)ws.items)[local / WG_PER_ITEM];
  const int line = (int)(local % WG_PER_ITEM) * 256 + threadIdx.x;
  if (line >= LINES) return;
  const cpx<T>* const in = it.tmp + line;
  T zr[B], zi[B], Zr[P], Zi[P];
#pragma unroll
  for (int z = 0; z < B; ++z) { const cpx<T> v = gld(in, (int64_t)z * LINES); zr[z] = v.x; zi[z] = v.y; }
  fwd_padded<B>(zr, zi, Zr, Zi);
  cpx<T>* const out = it.dst + line;
#pragma unroll
  for (int kz = 0; kz < P; ++kz) gst(out, (int64_t)kz * LINES, cpx<T>{Zr[kz], Zi[kz]});
}

// inverse z pass: one lane per (kx, ky) line, keep z < B2
template <int B2, typename T>
__global__ __launch_bounds__(256) void sup_inv_z(SetTable sets) {
  using Sh = SupShape<B2>;
  constexpr int P = Sh::P, B = B2;
  constexpr int LINES = Sh::PLANE;
  constexpr int WG_PER_ITEM = (LINES + 255) / 256;
  const int set = find_set(sets, blockIdx.x);
  const WorkSet& ws = sets.s[set];
  const int64_t local = blockIdx.x - ws.wg_begin;
  const SuperInvItem<T>& it = ((const SuperInvItem<T>*)ws.items)[local / WG_PER_ITEM];
  const int line = (int)(local % WG_PER_ITEM) * 256 + threadIdx.x;
  if (line >= LINES) return;
  const cpx<T>* const in = it.src + line;
  T Zr[P], Zi[P], zr[B], zi[B];
#pragma unroll
  for (int kz = 0; kz < P; ++kz) { const cpx<T> v = gld(in, (int64_t)kz * LINES); Zr[kz] = v.x; Zi[kz] = v.y; }
  inv_cropped<B>(Zr, Zi, zr, zi);
  cpx<T>* const out = it.tmp + line;
#pragma unroll
  for (int z = 0; z < B; ++z) gst(out, (int64_t)z * LINES, cpx<T>{zr[z], zi[z]});
}

// inverse (y, x) pass: one workgroup per (super-block, z-plane); crop, scale by 1/P^3 and write
// the children's cells.  LM = 0: plane z from the plane stack; LM = 1: from line-major planes.
template <int B2, typename T, typename TC, bool LM>
__global__ __launch_bounds__(64) void sup_inv_yx(SetTable sets) {
  using Sh = SupShape<B2>;
  constexpr int P = Sh::P, H = Sh::H, NB = Sh::NB;
  __shared__ cpx<T> pl[B2 * H];                 // [y][kx] after the y pass
  const int set = find_set(sets, blockIdx.x);
  const WorkSet& ws = sets.s[set];
  const int64_t local = blockIdx.x - ws.wg_begin;
  int64_t item;
  int z;
  if (!plane_of<B2, LM>(ws, local, &item, &z)) return;
  const SuperInvItem<T>& it = ((const SuperInvItem<T>*)ws.items)[item];
  const int tid = threadIdx.x;
  const cpx<T>* const in = LM ? it.tmp : it.tmp + (int64_t)z * Sh::PLANE;
  for (int kx = tid; kx < H; kx += 64) {
    T Yr[P], Yi[P], yr[B2], yi[B2];
#pragma unroll
    for (int ky = 0; ky < P; ++ky) {
      const cpx<T> v = LM ? gld(in, (int64_t)(ky * H + kx) * B2 + z) : gld(in, ky * H + kx);
      Yr[ky] = v.x;
      Yi[ky] = v.y;
    }
    inv_cropped<B2>(Yr, Yi, yr, yi);
#pragma unroll
    for (int y = 0; y < B2; ++y) pl[y * H + kx] = {yr[y], yi[y]};
  }
  __syncthreads();
  const T inv = T(1.0 / (double(P) * P * P));
  const int cz = z / NB, lz = z % NB;
  for (int y = tid; y < B2; y += 64) {
    T Xr[P], Xi[P], xr[B2], xi[B2];
#pragma unroll
    for (int k = 0; k < H; ++k) { Xr[k] = pl[y * H + k].x; Xi[k] = pl[y * H + k].y; }
#pragma unroll
    for (int k = 1; k < B2; ++k) { Xr[P - k] = Xr[k]; Xi[P - k] = -Xi[k]; }
    inv_cropped<B2>(Xr, Xi, xr, xi);
    const int cy = y / NB, ly = y % NB;
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      TC* c = (TC*)it.child[half + 2 * cy + 4 * cz];
      if (!c) continue;
      const gview<TC> row = gl(c + (lz * NB + ly) * NB);
#pragma unroll
      for (int x = 0; x < NB; ++x) row[x] = TC(xr[half * NB + x] * inv);
    }
  }
}

// workgroups of the line-major passes: B2 planes per item, items dealt to the 8 XCDs in turn
inline int64_t assign_wg_lm(SetTable& t, int B2) {
  int64_t wg = 0;
  for (int i = 0; i < t.n; ++i) {
    t.s[i].wg_begin = wg;
    wg += (t.s[i].count + 7) / 8 * 8 * (int64_t)B2;
  }
  return wg;
}

// kernel columns: one thread per (h, line, kz)
template <int B2, typename T>
__global__ __launch_bounds__(256) void kernel_columns_kernel(const cpx<T>* spec, cpx<T>* out) {
  using Sh = SupShape<B2>;
  constexpr int P = Sh::P;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (int64_t)14 * Sh::S) return;
  const int kz = (int)(i % P);
  const int64_t r = i / P;
  const int line = (int)(r % Sh::PLANE), h = (int)(r / Sh::PLANE);
  gst(out, i, gld(spec, (int64_t)h * Sh::S + (int64_t)kz * Sh::PLANE + line));
}

template <int B2, typename T, typename TC> hipError_t fwd_b2(SetTable& t, hipStream_t st, int mode) {
  using Sh = SupShape<B2>;
  if (mode == 1) {
    const int64_t wg = assign_wg_lm(t, B2);
    if (wg == 0) return hipSuccess;
    sup_fwd_xy<B2, T, TC, true><<<(unsigned)wg, 64, 0, st>>>(t);
    return hipGetLastError();
  }
  const int64_t wg1 = assign_wg(t, B2);
  if (wg1 == 0) return hipSuccess;
  sup_fwd_xy<B2, T, TC, false><<<(unsigned)wg1, 64, 0, st>>>(t);
  LGF_HIP_CHECK(hipGetLastError());
  const int64_t wg2 = assign_wg(t, (Sh::PLANE + 255) / 256);
  sup_fwd_z<B2, T><<<(unsigned)wg2, 256, 0, st>>>(t);
  return hipGetLastError();
}

template <int B2, typename T, typename TC> hipError_t inv_b2(SetTable& t, hipStream_t st, int mode) {
  using Sh = SupShape<B2>;
  if (mode == 1) {
    const int64_t wg = assign_wg_lm(t, B2);
    if (wg == 0) return hipSuccess;
    sup_inv_yx<B2, T, TC, true><<<(unsigned)wg, 64, 0, st>>>(t);
    return hipGetLastError();
  }
  const int64_t wg1 = assign_wg(t, (Sh::PLANE + 255) / 256);
  if (wg1 == 0) return hipSuccess;
  sup_inv_z<B2, T><<<(unsigned)wg1, 256, 0, st>>>(t);
  LGF_HIP_CHECK(hipGetLastError());
  const int64_t wg2 = assign_wg(t, B2);
  sup_inv_yx<B2, T, TC, false><<<(unsigned)wg2, 64, 0, st>>>(t);
  return hipGetLastError();
}

}  // namespace

// nb is the child block side; the super-block side is 2 nb.  T: transform type, TC: child type.
template <typename T, typename TC> hipError_t launch_super_fwd(int nb, SetTable& t, hipStream_t st, int mode) {
  if (mode != 0 && mode != 1) return hipErrorInvalidValue;
  if (nb == 16) return fwd_b2<32, T, TC>(t, st, mode);
  if (nb == 8) return fwd_b2<16, T, TC>(t, st, mode);
  return hipErrorInvalidValue;
}
template <typename T, typename TC> hipError_t launch_super_inv(int nb, SetTable& t, hipStream_t st, int mode) {
  if (mode != 0 && mode != 1) return hipErrorInvalidValue;
  if (nb == 16) return inv_b2<32, T, TC>(t, st, mode);
  if (nb == 8) return inv_b2<16, T, TC>(t, st, mode);
  return hipErrorInvalidValue;
}

template <typename T> hipError_t launch_kernel_columns(int nb, const cpx<T>* spectra, cpx<T>* out, hipStream_t st) {
  if (nb != 8 && nb != 16) return hipErrorInvalidValue;
  const int64_t n = (int64_t)14 * (nb == 16 ? SupShape<32>::S : SupShape<16>::S);
  const unsigned g = (unsigned)((n + 255) / 256);
  if (nb == 16) kernel_columns_kernel<32, T><<<g, 256, 0, st>>>(spectra, out);
  else kernel_columns_kernel<16, T><<<g, 256, 0, st>>>(spectra, out);
  return hipGetLastError();
}

template hipError_t launch_super_fwd<float, float>(int, SetTable&, hipStream_t, int);
template hipError_t launch_super_fwd<double, double>(int, SetTable&, hipStream_t, int);
template hipError_t launch_super_fwd<double, float>(int, SetTable&, hipStream_t, int);
template hipError_t launch_super_inv<float, float>(int, SetTable&, hipStream_t, int);
template hipError_t launch_super_inv<double, double>(int, SetTable&, hipStream_t, int);
template hipError_t launch_super_inv<double, float>(int, SetTable&, hipStream_t, int);
template hipError_t launch_kernel_columns<float>(int, const c32*, c32*, hipStream_t);
template hipError_t launch_kernel_columns<double>(int, const c64*, c64*, hipStream_t);

}  // namespace lgf
