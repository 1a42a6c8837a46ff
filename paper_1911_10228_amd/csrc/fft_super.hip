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

// P-th roots of unity e^{-2 pi i m / P} in global memory (read with vector loads: a lane's
// twiddles depend on its position in the line)
template <int P, typename T> struct Roots {
  cpx<T> w[P];
  constexpr Roots() : w{} {
    for (int m = 0; m < P; ++m) w[m] = cpx<T>{T(turn_cos(m, P)), T(-turn_sin(m, P))};
  }
};
template <int P, typename T> __device__ const Roots<P, T> kRoots{};
template <int P, typename T> __device__ __forceinline__ cpx<T> root(int m) {
  const gview<const T> r = gl((const T*)&kRoots<P, T>.w[0]);
  return {r[2 * m], r[2 * m + 1]};
}

// (item, first z-plane) of a workgroup that transforms ZP consecutive planes.  Plane-major
// (LM = 0, ZP = 1): consecutive workgroups take consecutive planes.  Line-major (LM = 1): every
// plane group of an item runs on one XCD (workgroup w goes to XCD w mod 8; set starts are
// multiples of 8), so the groups' pieces of each line meet in that XCD's L2 and leave it as
// whole lines.
template <int B2, bool LM, int ZP>
__device__ __forceinline__ bool plane_of(const WorkSet& ws, int64_t local, int64_t* item, int* z0) {
  if constexpr (!LM) {
    *item = local / B2;
    *z0 = (int)(local % B2);
    return true;
  }
  constexpr int G = B2 / ZP;
  const int64_t r = local >> 3;
  *z0 = (int)(r % G) * ZP;
  *item = (r / G) * 8 + (local & 7);
  return *item < ws.count;
}

// The (x, y) passes: one workgroup of 8 B2 threads per (super-block, z-plane), every length-P
// line (P = 2 B2 = 8 Q) split over Q or 8 lanes, with LDS exchanges between the two stages of
// each direction and between the directions.  Forward, zero-padded (n < B2 nonzero), with
// n = Q n1 + n2 and k = k1 + 8 k2:
//   Y[n2][k1] = W_P^{n2 k1} sum_{n1 < 4} x[Q n1 + n2] W_8^{n1 k1}     (lane n2)
//   X[k1 + 8 k2] = sum_{n2 < Q} Y[n2][k1] W_Q^{n2 k2}                 (lane k1)
// Inverse, cropped to n < B2, with k = Q k1 + k2 and n = n1 + 8 n2:
//   Z[k2][n1] = W_P^{-n1 k2} sum_{k1 < 8} X[Q k1 + k2] W_8^{-n1 k1}  (lane k2)
//   x[n1 + 8 n2] = sum_{k2 < Q} Z[k2][n1] W_Q^{-n2 k2}, n2 < Q / 2    (lane n1)
// The half spectrum along x of a real plane has B2 + 1 columns; columns kx = 0 and kx = B2 hold
// real values along y before the y transform, so they travel as one complex column
// (kx = 0 real, kx = B2 imaginary), and B2 columns fill the 8 B2 lanes.  Their y transforms are
// separated with the conjugate symmetry of the transform of a real sequence; on the way back the
// inverse y transform of that packed column is g0 + i g_B2 with both parts real.
//
// LDS: an exchange buffer E[line][m] (m = 8 n2 + k1 or 8 k2 + n1, one pad after every 8
// values) and the plane buffer between the directions, [column][y] forward and [y][column]
// inverse, each row swizzled by (row index mod 8): with these strides the accesses of every
// stage fall on distinct banks (one 2-way case: the mirrored reads of the inverse x stage).
// FP64: the two buffers share their space (two more barriers, twice the workgroups per CU).
//
// Line-major planes hold the B2 z values of a line contiguously, so a workgroup transforms ZP
// consecutive planes (8 B2 threads and one buffer set per plane) and the stage that touches
// the planes (the forward's last, the inverse's first) puts the plane index in the low lane
// bits: one memory instruction then moves ZP contiguous values of each of 64 / ZP lines
// instead of one value of each of 64 lines.  The per-plane buffers are NPL entries apart with
// NPL = W / ZP mod W, where W is the number of entries the LDS serves per cycle: 256 bytes for
// reads (the forward's stage reads the buffers), 128 bytes for writes (the inverse's writes
// them; the bank-conflict counter shows it), so the ZP planes' accesses of that stage take
// distinct banks as well.
template <int B2, typename T> struct XyShape {
  static constexpr int P = 2 * B2, Q = P / 8, H = B2 + 1, NB = B2 / 2, NT = 8 * B2;
  static constexpr int RS = 9 * Q;               // exchange row: 8 Q values and Q pads
  static constexpr int CS = B2 + 8;              // plane buffer row
  static constexpr bool ALIAS = sizeof(T) == 8;
  static constexpr int NE = B2 * RS, NP = B2 * CS;
  static constexpr int NLDS = ALIAS ? (NE > NP ? NE : NP) : NE + NP;
  template <int ZP, int BYTES> static constexpr int npl() {
    constexpr int W = BYTES / (int)sizeof(cpx<T>);
    return ZP == 1 ? NLDS : (NLDS + W - 1) / W * W + W / ZP;
  }
  static_assert(P == 8 * Q && (Q == 4 || Q == 8), "line shape");
};
// planes per workgroup of the line-major passes.  FP32: 4 (1024 threads, 115 KB of LDS).
// FP64: 2 (512 threads, 74 KB): alone the passes are faster with 4 planes (148 KB, one
// workgroup per CU: forward 24.5 against 25.7 us, inverse 28.0 against 33.3 us on 64
// super-blocks of 32^3), but in the solve they share the CUs with the far field's kernels,
// which fit beside a 74 KB workgroup and not beside a 148 KB one (FP64 solve of the
// 8^3 x 16^3 workload 0.206 -> 0.202 ms; one plane per workgroup 0.211 ms; four planes in the
// inverse only: the pass 32.1 -> 27.4 us alone, the solve 0.191 -> 0.196 ms)
template <int B2, typename T> constexpr int kXyPlanes = sizeof(T) == 8 ? 2 : 4;
__device__ __forceinline__ int xat(int m) { return m + (m >> 3); }

// Between the two x stages a line's values move between the lanes that own the line: with
// Q = 8 those are lanes 8 y .. 8 y + 7 of one wavefront in both stages, and the wavefront's LDS
// operations complete in order, so ordering within the wavefront suffices.
template <int Q> __device__ __forceinline__ void line_sync() {
  if constexpr (Q == 8) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

template <int B2, typename T, typename TC, bool LM, int ZP>
__global__ __launch_bounds__(8 * B2 * ZP) void sup_fwd_xy(SetTable sets) {
  using X = XyShape<B2, T>;
  constexpr int P = X::P, Q = X::Q, H = X::H, NB = X::NB, RS = X::RS, CS = X::CS;
  constexpr int NPL = X::template npl<ZP, 256>();
  static_assert(LM || ZP == 1, "plane-major passes take one plane per workgroup");
  __shared__ cpx<T> lds[ZP * NPL];
  const int set = find_set(sets, blockIdx.x);
  const WorkSet& ws = sets.s[set];
  const int64_t local = blockIdx.x - ws.wg_begin;
  int64_t item;
  int z0;
  if (!plane_of<B2, LM, ZP>(ws, local, &item, &z0)) return;
  const SuperFwdItem<T>& it = ((const SuperFwdItem<T>*)ws.items)[item];
  // the x stages and the first y stage: plane z0 + threadIdx.x / (8 B2)
  const int t = threadIdx.x % (8 * B2);
  const int z = z0 + threadIdx.x / (8 * B2);
  cpx<T>* const E = lds + (threadIdx.x / (8 * B2)) * NPL;
  cpx<T>* const PL = X::ALIAS ? E : E + X::NE;
  const int cz = z / NB, lz = z % NB;
  // x stage 1: lane (y, n2), the row's real values x = Q n1 + n2 (x < NB: octant cx = 0)
  if (t < B2 * Q) {
    const int y = t / Q, n2 = t % Q;
    const int oc = 2 * (y / NB) + 4 * cz;
    const int off = (lz * NB + y % NB) * NB;
    T xr[4], xi[4], Yr[8], Yi[8];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const TC* c = child_ptr<TC>((const TC*)it.child[oc + h], it.child_in[oc + h], ws.in);
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        xr[2 * h + j] = c ? T(gl(c + off)[Q * j + n2]) : T(0);
        xi[2 * h + j] = T(0);
      }
    }
    fwd_padded<4>(xr, xi, Yr, Yi);
#pragma unroll
    for (int k1 = 0; k1 < 8; ++k1) {
      const cpx<T> w = k1 ? root<P, T>(n2 * k1) : cpx<T>{T(1), T(0)};
      E[y * RS + xat(8 * n2 + k1)] = cpx<T>{Yr[k1] * w.x - Yi[k1] * w.y, Yr[k1] * w.y + Yi[k1] * w.x};
    }
  }
  line_sync<Q>();              // the x stages: a line's 8 lanes in one wavefront
  // x stage 2: lane (y, k1); columns kx = k1 + 8 k2 <= B2 to the plane buffer [kx][y]
  {
    const int y = t >> 3, k1 = t & 7;
    T xr[Q], xi[Q];
#pragma unroll
    for (int n2 = 0; n2 < Q; ++n2) {
      const cpx<T> v = E[y * RS + xat(8 * n2 + k1)];
      xr[n2] = v.x;
      xi[n2] = v.y;
    }
    fft_inreg<Q, -1>(xr, xi);
    if constexpr (X::ALIAS) __syncthreads();
#pragma unroll
    for (int k2 = 0; k2 < Q / 2; ++k2) {
      const int c = k1 + 8 * k2;
      const cpx<T> v = c ? cpx<T>{xr[k2], xi[k2]} : cpx<T>{xr[0], xr[Q / 2]};   // kx = 0 | B2 packed
      PL[c * CS + (y ^ (c & 7))] = v;
    }
  }
  __syncthreads();
  // y stage 1: lane (c, n2), the column's values y = Q n1 + n2 (y < B2)
  T Yr[8], Yi[8];
  const bool y1 = t < B2 * Q;
  const int c1 = t / Q, m2 = t % Q;
  if (y1) {
    T vr[4], vi[4];
#pragma unroll
    for (int n1 = 0; n1 < 4; ++n1) {
      const cpx<T> v = PL[c1 * CS + ((Q * n1 + m2) ^ (c1 & 7))];
      vr[n1] = v.x;
      vi[n1] = v.y;
    }
    fwd_padded<4>(vr, vi, Yr, Yi);
  }
  if constexpr (X::ALIAS) __syncthreads();
  if (y1) {
#pragma unroll
    for (int k1 = 0; k1 < 8; ++k1) {
      const cpx<T> w = k1 ? root<P, T>(m2 * k1) : cpx<T>{T(1), T(0)};
      E[c1 * RS + xat(8 * m2 + k1)] = cpx<T>{Yr[k1] * w.x - Yi[k1] * w.y, Yr[k1] * w.y + Yi[k1] * w.x};
    }
  }
  __syncthreads();
  // y stage 2: lane (c, k1, plane), outputs ky = k1 + 8 k2 of plane z0 + zp
  const int zp = threadIdx.x % ZP, r = threadIdx.x / ZP;
  const int c = r >> 3, k1 = r & 7;
  const cpx<T>* const E2 = lds + zp * NPL;
  T zr[Q], zi[Q];
#pragma unroll
  for (int n2 = 0; n2 < Q; ++n2) {
    const cpx<T> v = E2[c * RS + xat(8 * n2 + k1)];
    zr[n2] = v.x;
    zi[n2] = v.y;
  }
  fft_inreg<Q, -1>(zr, zi);
  cpx<T>* const out = LM ? it.tmp : it.tmp + (int64_t)z0 * (P * H);
  auto put = [&](int ky, int kx, cpx<T> v) {
    if constexpr (LM) gst(out, (int64_t)(ky * H + kx) * B2 + z0 + zp, v);
    else gst(out, ky * H + kx, v);
  };
  if ((threadIdx.x >> 6) == 0) {
    // wave 0 holds the packed columns (c = 0: lanes below 8 ZP): A[ky] + i B[ky] with A, B the
    // transforms of the real columns kx = 0 and B2, so A[ky] = (Z[ky] + conj Z[-ky]) / 2 and
    // B[ky] = (Z[ky] - conj Z[-ky]) / 2i.  Z[-ky] of ky = k1 + 8 k2 is held by the lane of
    // 8 - k1 (k2' = Q - 1 - k2), or for k1 = 0 by the lane itself (k2' = (Q - k2) mod Q).
    T pr[Q], pi[Q];
    const int src = ((r & ~7) | ((8 - k1) & 7)) * ZP + zp;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      pr[j] = __shfl(zr[j], src);
      pi[j] = __shfl(zi[j], src);
    }
    if (c == 0) {
#pragma unroll
      for (int k2 = 0; k2 < Q; ++k2) {
        const T mr = k1 ? pr[Q - 1 - k2] : zr[(Q - k2) % Q];
        const T mi = k1 ? pi[Q - 1 - k2] : zi[(Q - k2) % Q];
        const int ky = k1 + 8 * k2;
        put(ky, 0, cpx<T>{T(0.5) * (zr[k2] + mr), T(0.5) * (zi[k2] - mi)});
        put(ky, B2, cpx<T>{T(0.5) * (zi[k2] + mi), T(0.5) * (mr - zr[k2])});
      }
      return;
    }
  }
#pragma unroll
  for (int k2 = 0; k2 < Q; ++k2) put(k1 + 8 * k2, c, cpx<T>{zr[k2], zi[k2]});
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

// inverse (y, x) pass: one workgroup per (super-block, z-plane) as the forward pass; crop,
// scale by 1/P^3 and write the children's cells.  LM = 0: plane z from the plane stack;
// LM = 1: from line-major planes.
template <int B2, typename T, typename TC, bool LM, int ZP>
__global__ __launch_bounds__(8 * B2 * ZP) void sup_inv_yx(SetTable sets) {
  using X = XyShape<B2, T>;
  constexpr int P = X::P, Q = X::Q, H = X::H, NB = X::NB, RS = X::RS, CS = X::CS;
  constexpr int NPL = X::template npl<ZP, 128>();
  static_assert(LM || ZP == 1, "plane-major passes take one plane per workgroup");
  __shared__ cpx<T> lds[ZP * NPL];
  const int set = find_set(sets, blockIdx.x);
  const WorkSet& ws = sets.s[set];
  const int64_t local = blockIdx.x - ws.wg_begin;
  int64_t item;
  int z0;
  if (!plane_of<B2, LM, ZP>(ws, local, &item, &z0)) return;
  const SuperInvItem<T>& it = ((const SuperInvItem<T>*)ws.items)[item];
  const cpx<T>* const in = LM ? it.tmp : it.tmp + (int64_t)z0 * (P * H);
  // y stage 1: lane (c, k2, plane), ky = Q k1 + k2 of plane z0 + zp; column 0 carries
  // kx = 0 + i kx = B2
  {
    const int zp = threadIdx.x % ZP, r = threadIdx.x / ZP;
    auto get = [&](int ky, int kx) {
      if constexpr (LM) return gld(in, (int64_t)(ky * H + kx) * B2 + z0 + zp);
      else return gld(in, ky * H + kx);
    };
    if (r < B2 * Q) {
      const int c = r / Q, k2 = r % Q;
      cpx<T>* const E1 = lds + zp * NPL;
      T zr[8], zi[8];
#pragma unroll
      for (int k1 = 0; k1 < 8; ++k1) {
        const int ky = Q * k1 + k2;
        cpx<T> v = get(ky, c);
        if (c == 0) {
          const cpx<T> b = get(ky, B2);
          v = cpx<T>{v.x - b.y, v.y + b.x};
        }
        zr[k1] = v.x;
        zi[k1] = v.y;
      }
      fft_inreg<8, +1>(zr, zi);
#pragma unroll
      for (int n1 = 0; n1 < 8; ++n1) {
        const cpx<T> w = n1 ? root<P, T>(n1 * k2) : cpx<T>{T(1), T(0)};   // conjugated below
        E1[c * RS + xat(8 * k2 + n1)] = cpx<T>{zr[n1] * w.x + zi[n1] * w.y, zi[n1] * w.x - zr[n1] * w.y};
      }
    }
  }
  // the remaining stages: plane z0 + threadIdx.x / (8 B2)
  const int t = threadIdx.x % (8 * B2);
  const int z = z0 + threadIdx.x / (8 * B2);
  cpx<T>* const E = lds + (threadIdx.x / (8 * B2)) * NPL;
  cpx<T>* const PL = X::ALIAS ? E : E + X::NE;
  __syncthreads();
  // y stage 2: lane (c, n1), y = n1 + 8 n2 < B2, to the plane buffer [y][c]
  {
    const int c = t >> 3, n1 = t & 7;
    T Zr[Q], Zi[Q], yr[Q / 2], yi[Q / 2];
#pragma unroll
    for (int k2 = 0; k2 < Q; ++k2) {
      const cpx<T> v = E[c * RS + xat(8 * k2 + n1)];
      Zr[k2] = v.x;
      Zi[k2] = v.y;
    }
    inv_cropped<Q / 2>(Zr, Zi, yr, yi);
    if constexpr (X::ALIAS) __syncthreads();
#pragma unroll
    for (int n2 = 0; n2 < Q / 2; ++n2) {
      const int y = n1 + 8 * n2;
      PL[y * CS + (c ^ (y & 7))] = cpx<T>{yr[n2], yi[n2]};
    }
  }
  __syncthreads();
  // x stage 1: lane (y, k2), kx = Q k1 + k2 over the full line (kx > B2 from the conjugates)
  T Xr[8], Xi[8];
  const bool x1 = t < B2 * Q;
  const int y1 = t / Q, m2 = t % Q;
  if (x1) {
#pragma unroll
    for (int k1 = 0; k1 < 8; ++k1) {
      int col = k1 < 4 ? Q * k1 + m2 : Q * (8 - k1) - m2;
      col = col == B2 ? 0 : col;
      const cpx<T> v = PL[y1 * CS + (col ^ (y1 & 7))];
      if ((k1 == 0 || k1 == 4) && m2 == 0) {
        Xr[k1] = k1 == 0 ? v.x : v.y;                // the real columns kx = 0 and B2
        Xi[k1] = T(0);
      } else {
        Xr[k1] = v.x;
        Xi[k1] = k1 < 4 ? v.y : -v.y;
      }
    }
    fft_inreg<8, +1>(Xr, Xi);
  }
  if constexpr (X::ALIAS) __syncthreads();
  if (x1) {
#pragma unroll
    for (int n1 = 0; n1 < 8; ++n1) {
      const cpx<T> w = n1 ? root<P, T>(n1 * m2) : cpx<T>{T(1), T(0)};
      E[y1 * RS + xat(8 * m2 + n1)] = cpx<T>{Xr[n1] * w.x + Xi[n1] * w.y, Xi[n1] * w.x - Xr[n1] * w.y};
    }
  }
  line_sync<Q>();              // the x stages: a line's 8 lanes in one wavefront
  // x stage 2: lane (y, n1), x = n1 + 8 n2 < B2 (real part), scaled, to the children
  const int y = t >> 3, n1 = t & 7;
  T Zr[Q], Zi[Q], xr[Q / 2], xi[Q / 2];
#pragma unroll
  for (int k2 = 0; k2 < Q; ++k2) {
    const cpx<T> v = E[y * RS + xat(8 * k2 + n1)];
    Zr[k2] = v.x;
    Zi[k2] = v.y;
  }
  inv_cropped<Q / 2>(Zr, Zi, xr, xi);
  const T inv = T(1.0 / (double(P) * P * P));
  const int cz = z / NB, lz = z % NB, cy = y / NB, ly = y % NB;
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    TC* ch = (TC*)it.child[half + 2 * cy + 4 * cz];
    if (!ch) continue;
    const gview<TC> row = gl(ch + (lz * NB + ly) * NB);
#pragma unroll
    for (int j = 0; j < Q / 4; ++j) row[n1 + 8 * j] = TC(xr[half * (Q / 4) + j] * inv);
  }
}

// workgroups of the line-major passes: `groups` plane groups per item, items dealt to the 8 XCDs
// in turn
inline int64_t assign_wg_lm(SetTable& t, int groups) {
  int64_t wg = 0;
  for (int i = 0; i < t.n; ++i) {
    t.s[i].wg_begin = wg;
    wg += (t.s[i].count + 7) / 8 * 8 * (int64_t)groups;
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
    constexpr int ZP = kXyPlanes<B2, T>;
    const int64_t wg = assign_wg_lm(t, B2 / ZP);
    if (wg == 0) return hipSuccess;
    sup_fwd_xy<B2, T, TC, true, ZP><<<(unsigned)wg, 8 * B2 * ZP, 0, st>>>(t);
    return hipGetLastError();
  }
  const int64_t wg1 = assign_wg(t, B2);
  if (wg1 == 0) return hipSuccess;
  sup_fwd_xy<B2, T, TC, false, 1><<<(unsigned)wg1, 8 * B2, 0, st>>>(t);
  LGF_HIP_CHECK(hipGetLastError());
  const int64_t wg2 = assign_wg(t, (Sh::PLANE + 255) / 256);
  sup_fwd_z<B2, T><<<(unsigned)wg2, 256, 0, st>>>(t);
  return hipGetLastError();
}

template <int B2, typename T, typename TC> hipError_t inv_b2(SetTable& t, hipStream_t st, int mode) {
  using Sh = SupShape<B2>;
  if (mode == 1) {
    constexpr int ZP = kXyPlanes<B2, T>;
    const int64_t wg = assign_wg_lm(t, B2 / ZP);
    if (wg == 0) return hipSuccess;
    sup_inv_yx<B2, T, TC, true, ZP><<<(unsigned)wg, 8 * B2 * ZP, 0, st>>>(t);
    return hipGetLastError();
  }
  const int64_t wg1 = assign_wg(t, (Sh::PLANE + 255) / 256);
  if (wg1 == 0) return hipSuccess;
  sup_inv_z<B2, T><<<(unsigned)wg1, 256, 0, st>>>(t);
  LGF_HIP_CHECK(hipGetLastError());
  const int64_t wg2 = assign_wg(t, B2);
  sup_inv_yx<B2, T, TC, false, 1><<<(unsigned)wg2, 8 * B2, 0, st>>>(t);
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
