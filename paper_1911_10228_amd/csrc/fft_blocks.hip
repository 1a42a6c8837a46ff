// Zero-padded block FFTs of the block convolution (Sec. 2.1: each block convolution is a
// Hadamard product in Fourier space of the zero-padded block and kernel).
//
// Forward: n_b^3 real block, padded to P^3 (P = 2 n_b), real-to-complex along x, complex along
// y and z.  Only the nonzero half of every line is read, so each length-P transform is two
// length-n_b transforms (even and twiddled odd outputs).  Inverse: the mirror image, and only the
// first n_b outputs of every line are formed (the crop of the linear convolution).
//
// One workgroup transforms BPW blocks; each lane holds one line in registers; the three passes
// are separated by LDS transposes in the layouts A[b][z][y][kx] (after x) and B[b][z][ky][kx]
// (after y).  A and B share the LDS region; every lane stages its line in registers across a
// barrier before the overlapping write.
#include "kernels.hpp"

namespace lgf {

namespace {

template <int NB> struct FftShape {
  static constexpr int P = 2 * NB;
  static constexpr int H = NB + 1;              // kx in [0, NB]
  static constexpr int BPW = NB == 16 ? 1 : 4;  // blocks per workgroup
  static constexpr int YL = BPW * NB * H;       // y-pass lines
  static constexpr int NT = (YL + 63) / 64 * 64;
  static constexpr int LDS = BPW * NB * P * H;  // complex entries
  static constexpr int S = P * P * H;
};

template <int NB, typename T>
__global__ __launch_bounds__(FftShape<NB>::NT) void fft_fwd_kernel(SetTable sets) {
  using Sh = FftShape<NB>;
  constexpr int P = Sh::P, H = Sh::H, BPW = Sh::BPW, NT = Sh::NT;
  __shared__ cpx<T> lds[Sh::LDS];
  const int set = find_set(sets, blockIdx.x);
  const WorkSet& ws = sets.s[set];
  const FftFwdItem<T>* items = (const FftFwdItem<T>*)ws.items;
  const int first = (int)(blockIdx.x - ws.wg_begin) * BPW;
  const int tid = threadIdx.x;

  // x pass: lines (b, z, y)
  for (int l = tid; l < BPW * NB * NB; l += NT) {
    const int y = l % NB, z = (l / NB) % NB, b = l / (NB * NB);
    if (first + b >= ws.count) continue;
    const gview<const T> src = gl(items[first + b].src + (z * NB + y) * NB);
    T xr[NB], xi[NB], Xr[P], Xi[P];
#pragma unroll
    for (int x = 0; x < NB; ++x) { xr[x] = src[x]; xi[x] = T(0); }
    fwd_padded<NB>(xr, xi, Xr, Xi);
    cpx<T>* a = lds + ((b * NB + z) * NB + y) * H;
#pragma unroll
    for (int k = 0; k < H; ++k) a[k] = {Xr[k], Xi[k]};
  }
  __syncthreads();

  // y pass: lines (b, z, kx), staged in registers (A and B overlap)
  T yr[NB], yi[NB];
  const int yl = tid;
  const int kx = yl % H, z = (yl / H) % NB, b = yl / (H * NB);
  const bool yact = yl < Sh::YL;
  if (yact) {
#pragma unroll
    for (int y = 0; y < NB; ++y) {
      const cpx<T> v = lds[((b * NB + z) * NB + y) * H + kx];
      yr[y] = v.x; yi[y] = v.y;
    }
  }
  __syncthreads();
  if (yact) {
    T Yr[P], Yi[P];
    fwd_padded<NB>(yr, yi, Yr, Yi);
#pragma unroll
    for (int ky = 0; ky < P; ++ky) lds[((b * NB + z) * P + ky) * H + kx] = {Yr[ky], Yi[ky]};
  }
  __syncthreads();

  // z pass: lines (b, ky, kx) -> global [kz][ky][kx]
  for (int l = tid; l < BPW * P * H; l += NT) {
    const int kxx = l % H, ky = (l / H) % P, bb = l / (H * P);
    if (first + bb >= ws.count) continue;
    T zr[NB], zi[NB], Zr[P], Zi[P];
#pragma unroll
    for (int zz = 0; zz < NB; ++zz) {
      const cpx<T> v = lds[((bb * NB + zz) * P + ky) * H + kxx];
      zr[zz] = v.x; zi[zz] = v.y;
    }
    fwd_padded<NB>(zr, zi, Zr, Zi);
    cpx<T>* const dst = items[first + bb].dst + ky * H + kxx;
#pragma unroll
    for (int kz = 0; kz < P; ++kz) gst(dst, kz * P * H, cpx<T>{Zr[kz], Zi[kz]});
  }
}

// Forward transform of 16^3 blocks split over 4 workgroups per block by kx (groups of 5, 4, 4
// and 4 of the 17 half-spectrum columns): each workgroup runs the x pass of every row (keeping
// its columns; the rows are read from the XCD's L2 after the first workgroup), then the y and z
// passes of its columns only.  So a level of 64 blocks is 256 workgroups instead of 64, and each
// workgroup's y and z passes are a quarter as long.  Workgroup w of a set takes block
// 8 (w / 32) + w mod 8, group (w / 8) mod 4: the groups of a block share one XCD.
template <typename T>
__global__ __launch_bounds__(256) void fft_fwd16_split_kernel(SetTable sets) {
  constexpr int NB = 16, P = 32, H = 17, KW = 5;
  __shared__ cpx<T> lds[NB * P * KW];            // after x: A[z][y][j]; after y: B[z][ky][j]
  const int set = find_set(sets, blockIdx.x);
  const WorkSet& ws = sets.s[set];
  const int64_t local = blockIdx.x - ws.wg_begin;
  const int64_t item = (local >> 5) * 8 + (local & 7);
  if (item >= ws.count) return;
  const int g = (int)((local >> 3) & 3);
  const int k0 = g == 0 ? 0 : 1 + 4 * g, kw = g == 0 ? 5 : 4;
  const FftFwdItem<T>& it = ((const FftFwdItem<T>*)ws.items)[item];
  const int tid = threadIdx.x;
  // x pass: row (z, y) = tid
  {
    const int y = tid % NB, z = tid / NB;
    const gview<const T> src = gl(it.src + (z * NB + y) * NB);
    T xr[NB], xi[NB], Xr[P], Xi[P];
#pragma unroll
    for (int x = 0; x < NB; ++x) { xr[x] = src[x]; xi[x] = T(0); }
    fwd_padded<NB>(xr, xi, Xr, Xi);
#pragma unroll
    for (int j = 0; j < KW; ++j) {
      // compile-time register index: select the group's column k0 + j among the candidates
      cpx<T> v{T(0), T(0)};
#pragma unroll
      for (int gg = 0; gg < 4; ++gg) {
        const int kk = (gg == 0 ? 0 : 1 + 4 * gg) + j;
        if (gg == g && kk < H) v = cpx<T>{Xr[kk], Xi[kk]};
      }
      if (j < kw) lds[(z * NB + y) * KW + j] = v;
    }
  }
  __syncthreads();
  // y pass: line (z, j), staged in registers (A and B overlap)
  const bool yact = tid < NB * kw;
  const int yz = tid / kw, yj = tid % kw;
  T yr[NB], yi[NB];
  if (yact) {
#pragma unroll
    for (int y = 0; y < NB; ++y) {
      const cpx<T> v = lds[(yz * NB + y) * KW + yj];
      yr[y] = v.x;
      yi[y] = v.y;
    }
  }
  __syncthreads();
  if (yact) {
    T Yr[P], Yi[P];
    fwd_padded<NB>(yr, yi, Yr, Yi);
#pragma unroll
    for (int ky = 0; ky < P; ++ky) lds[(yz * P + ky) * KW + yj] = {Yr[ky], Yi[ky]};
  }
  __syncthreads();
  // z pass: line (ky, j) -> global [kz][ky][k0 + j]
  if (tid < P * kw) {
    const int ky = tid / kw, j = tid % kw;
    T zr[NB], zi[NB], Zr[P], Zi[P];
#pragma unroll
    for (int z = 0; z < NB; ++z) {
      const cpx<T> v = lds[(z * P + ky) * KW + j];
      zr[z] = v.x;
      zi[z] = v.y;
    }
    fwd_padded<NB>(zr, zi, Zr, Zi);
    cpx<T>* const dst = it.dst + ky * H + k0 + j;
#pragma unroll
    for (int kz = 0; kz < P; ++kz) gst(dst, kz * P * H, cpx<T>{Zr[kz], Zi[kz]});
  }
}

template <int NB, typename T>
__global__ __launch_bounds__(FftShape<NB>::NT) void fft_inv_kernel(SetTable sets) {
  using Sh = FftShape<NB>;
  constexpr int P = Sh::P, H = Sh::H, BPW = Sh::BPW, NT = Sh::NT;
  __shared__ cpx<T> lds[Sh::LDS];
  const int set = find_set(sets, blockIdx.x);
  const WorkSet& ws = sets.s[set];
  const FftInvItem<T>* items = (const FftInvItem<T>*)ws.items;
  const int first = (int)(blockIdx.x - ws.wg_begin) * BPW;
  const int tid = threadIdx.x;

  // z pass: lines (b, ky, kx) from global, keep z < NB -> B[b][z][ky][kx]
  for (int l = tid; l < BPW * P * H; l += NT) {
    const int kx = l % H, ky = (l / H) % P, b = l / (H * P);
    if (first + b >= ws.count) continue;
    const cpx<T>* const src = items[first + b].src + ky * H + kx;
    T Zr[P], Zi[P], zr[NB], zi[NB];
#pragma unroll
    for (int kz = 0; kz < P; ++kz) {
      const cpx<T> v = gld(src, kz * P * H);
      Zr[kz] = v.x; Zi[kz] = v.y;
    }
    inv_cropped<NB>(Zr, Zi, zr, zi);
#pragma unroll
    for (int z = 0; z < NB; ++z) lds[((b * NB + z) * P + ky) * H + kx] = {zr[z], zi[z]};
  }
  __syncthreads();

  // y pass: lines (b, z, kx) staged in registers, keep y < NB -> A[b][z][y][kx]
  T Yr[P], Yi[P];
  const int yl = tid;
  const int kx = yl % H, z = (yl / H) % NB, b = yl / (H * NB);
  const bool yact = yl < Sh::YL;
  if (yact) {
#pragma unroll
    for (int ky = 0; ky < P; ++ky) {
      const cpx<T> v = lds[((b * NB + z) * P + ky) * H + kx];
      Yr[ky] = v.x; Yi[ky] = v.y;
    }
  }
  __syncthreads();
  if (yact) {
    T yr[NB], yi[NB];
    inv_cropped<NB>(Yr, Yi, yr, yi);
#pragma unroll
    for (int y = 0; y < NB; ++y) lds[((b * NB + z) * NB + y) * H + kx] = {yr[y], yi[y]};
  }
  __syncthreads();

  // x pass: lines (b, z, y): Hermitian completion of kx, complex inverse, real part / P^3
  const T inv = T(1.0 / (double(P) * P * P));
  for (int l = tid; l < BPW * NB * NB; l += NT) {
    const int y = l % NB, zz = (l / NB) % NB, bb = l / (NB * NB);
    if (first + bb >= ws.count) continue;
    const cpx<T>* a = lds + ((bb * NB + zz) * NB + y) * H;
    T Xr[P], Xi[P], xr[NB], xi[NB];
#pragma unroll
    for (int k = 0; k < H; ++k) {
      const cpx<T> v = a[k];
      Xr[k] = v.x; Xi[k] = v.y;
    }
#pragma unroll
    for (int k = 1; k < NB; ++k) { Xr[P - k] = Xr[k]; Xi[P - k] = -Xi[k]; }
    inv_cropped<NB>(Xr, Xi, xr, xi);
    const gview<T> dst = gl(items[first + bb].dst + (zz * NB + y) * NB);
#pragma unroll
    for (int x = 0; x < NB; ++x) dst[x] = xr[x] * inv;
  }
}

template <int NB, typename T> hipError_t fwd_nb(SetTable& t, hipStream_t st) {
  using Sh = FftShape<NB>;
  if constexpr (NB == 16) {                    // 4 workgroups per block (see fft_fwd16_split_kernel)
    int64_t wg = 0;
    for (int i = 0; i < t.n; ++i) {
      t.s[i].wg_begin = wg;
      wg += (t.s[i].count + 7) / 8 * 32;
    }
    if (wg == 0) return hipSuccess;
    fft_fwd16_split_kernel<T><<<(unsigned)wg, 256, 0, st>>>(t);
    return hipGetLastError();
  }
  const int64_t wg = assign_wg(t, 1, Sh::BPW);
  if (wg == 0) return hipSuccess;
  fft_fwd_kernel<NB, T><<<(unsigned)wg, Sh::NT, 0, st>>>(t);
  return hipGetLastError();
}
template <int NB, typename T> hipError_t inv_nb(SetTable& t, hipStream_t st) {
  using Sh = FftShape<NB>;
  const int64_t wg = assign_wg(t, 1, Sh::BPW);
  if (wg == 0) return hipSuccess;
  fft_inv_kernel<NB, T><<<(unsigned)wg, Sh::NT, 0, st>>>(t);
  return hipGetLastError();
}

}  // namespace

template <typename T> hipError_t launch_fft_fwd(int nb, SetTable& t, hipStream_t st) {
  if (nb == 16) return fwd_nb<16, T>(t, st);
  if (nb == 8) return fwd_nb<8, T>(t, st);
  return hipErrorInvalidValue;
}
template <typename T> hipError_t launch_fft_inv(int nb, SetTable& t, hipStream_t st) {
  if (nb == 16) return inv_nb<16, T>(t, st);
  if (nb == 8) return inv_nb<8, T>(t, st);
  return hipErrorInvalidValue;
}

template hipError_t launch_fft_fwd<float>(int, SetTable&, hipStream_t);
template hipError_t launch_fft_fwd<double>(int, SetTable&, hipStream_t);
template hipError_t launch_fft_inv<float>(int, SetTable&, hipStream_t);
template hipError_t launch_fft_inv<double>(int, SetTable&, hipStream_t);

}  // namespace lgf
