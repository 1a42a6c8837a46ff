// Block-local operators of the FLGF and of the block-refined scheme:
//   * anterpolation R = J^T (upward pass) and interpolation J (downward pass) with Lagrange
//     weights on the block grid (Sec. 2.1, Algorithm 1, steps 1 and 3), separable, staged in LDS;
//   * coarsening C: average of the 2x2x2 child cells (Sec. 3, regularization);
//   * quadratic refinement J^l of the parent's leaf-only field onto a child block and the source
//     correction g = f - L^l(J^l w^l) (Sec. 3, Algorithm 2, step 2b, reading: the operator acts
//     on the interpolated field); neighbour values come from the adjacent same-level block, or,
//     where there is none, from the parent's quadratic extended one child cell outward;
//   * FP64 residual r = f - L^l u of defect correction (the update u += e is the correction
//     pass's combine in accumulate mode).
// The 1-D weight tables are computed on the host in FP64.
#include "kernels.hpp"

namespace lgf {

namespace {

constexpr int kOpThreads = 256;

// Block kernels give each thread the cells i = tid + j kOpThreads, j < N3 / kOpThreads, and
// load all of a thread's values into registers before the first store: the block pointers are
// generic, so the compiler may not move a load past an earlier store, and a load-store loop
// would wait one memory round trip per cell.
template <int NB> constexpr int per_thread() { return NB * NB * NB / kOpThreads; }


// child += (Wz (x) Wy (x) Wx) parent for octant c; W is [2 NB][NB] row-major (FP64).
// Arithmetic in the parent's type TP, stored in the child's type TC.  The passes work in place
// on one block-sized LDS array (each thread holds its pass outputs in registers across a
// barrier): 38 KB in FP64, so that the kernel fits on a CU beside the inverse (y, x) pass of
// the super-block transforms, with which it shares the GPU at the end of a solve.
template <int NB, typename TC, typename TP>
__global__ __launch_bounds__(kOpThreads) void interp_kernel(SetTable sets) {
  using T = TP;
  constexpr int N3 = NB * NB * NB;
  __shared__ T b0[N3];
  __shared__ T w[3][NB][NB];
  const int set = find_set(sets, blockIdx.x);
  const WorkSet& ws = sets.s[set];
  const InterpItem<TC, TP>& it = ((const InterpItem<TC, TP>*)ws.items)[blockIdx.x - ws.wg_begin];
  const gview<const double> __restrict__ W = gl(ws.w);
  const int c[3] = {it.octant & 1, (it.octant >> 1) & 1, (it.octant >> 2) & 1};
  constexpr int PT = per_thread<NB>();
  {
    TP pv[PT];
#pragma unroll
    for (int j = 0; j < PT; ++j) pv[j] = gl(it.parent)[threadIdx.x + j * kOpThreads];
#pragma unroll
    for (int j = 0; j < PT; ++j) b0[threadIdx.x + j * kOpThreads] = pv[j];
  }
  TC cv[PT];
  if (it.accumulate) {
#pragma unroll
    for (int j = 0; j < PT; ++j) cv[j] = gl(it.child)[threadIdx.x + j * kOpThreads];
  }
  for (int i = threadIdx.x; i < 3 * NB * NB; i += kOpThreads) {
    const int d = i / (NB * NB), r = (i / NB) % NB, m = i % NB;
    w[d][r][m] = T(W[(c[d] * NB + r) * NB + m]);
  }
  __syncthreads();
  // x and y passes: a thread's output X (x pass) and Y (y pass) are the same for all its cells
  // (kOpThreads is a multiple of NB^2), so its weight row is read once; its cells' sums are
  // unrolled so that their multiply-add chains interleave
  static_assert(kOpThreads % (NB * NB) == 0, "thread layout");
  {
    T wr[NB];
#pragma unroll
    for (int x = 0; x < NB; ++x) wr[x] = w[0][threadIdx.x % NB][x];
    T o[PT];
#pragma unroll
    for (int j = 0; j < PT; ++j) {                               // x
      const int i = threadIdx.x + j * kOpThreads, yz = i / NB;
      T s = 0;
#pragma unroll
      for (int x = 0; x < NB; ++x) s += wr[x] * b0[yz * NB + x];
      o[j] = s;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < PT; ++j) b0[threadIdx.x + j * kOpThreads] = o[j];
  }
  __syncthreads();
  {
    T wr[NB];
#pragma unroll
    for (int y = 0; y < NB; ++y) wr[y] = w[1][(threadIdx.x / NB) % NB][y];
    T o[PT];
#pragma unroll
    for (int j = 0; j < PT; ++j) {                               // y
      const int i = threadIdx.x + j * kOpThreads, X = i % NB, z = i / (NB * NB);
      T s = 0;
#pragma unroll
      for (int y = 0; y < NB; ++y) s += wr[y] * b0[(z * NB + y) * NB + X];
      o[j] = s;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < PT; ++j) b0[threadIdx.x + j * kOpThreads] = o[j];
  }
  __syncthreads();
  const gview<TC> child = gl(it.child);
  const bool accumulate = it.accumulate;
  TC out[PT];
#pragma unroll
  for (int j = 0; j < PT; ++j) {                              // z
    const int i = threadIdx.x + j * kOpThreads;
    const int XY = i % (NB * NB), Z = i / (NB * NB);
    T s = 0;
#pragma unroll
    for (int z = 0; z < NB; ++z) s += w[2][Z][z] * b0[z * NB * NB + XY];
    out[j] = TC(accumulate ? T(cv[j]) + s : s);
  }
#pragma unroll
  for (int j = 0; j < PT; ++j) child[threadIdx.x + j * kOpThreads] = out[j];
}

// parent = sum_c (Wz (x) Wy (x) Wx)^T child_c, arithmetic in the parent's type TP.
// One workgroup computes a slab of NB/8 parent z-planes: the z pass comes first (it mixes child
// planes into the slab's parent planes), so the y and x passes of different slabs are
// independent and eight workgroups share a parent without redundant arithmetic.  By linearity
// the children are summed as early as their weights allow: after the z pass per (cx, cy) (the
// two cz children), after the y pass per cx, so the passes run on 8, 4 and 2 arrays with three
// barriers in all.
template <int NB, typename TC, typename TP>
__global__ __launch_bounds__(NB * NB) void anterp_kernel(SetTable sets) {
  using T = TP;
  constexpr int SL = NB / 8;           // parent z-planes per workgroup
  __shared__ T w[2][NB][NB];           // w[c][r][m] = W[c NB + r][m]
  __shared__ T t1[4][SL][NB][NB];      // z pass, per (cx, cy): [z][Y][X]
  __shared__ T t2[2][SL][NB][NB];      // y pass, per cx: [z][y][X]
  const int set = find_set(sets, blockIdx.x);
  const WorkSet& ws = sets.s[set];
  // workgroup w of the set: parent 8 (w / 64) + w mod 8, slab (w / 8) mod 8, so that the eight
  // slabs of a parent run on one XCD (workgroups go to the XCDs in turn; set starts are
  // multiples of 64) and read its children once from HBM into that XCD's L2
  const int64_t local = blockIdx.x - ws.wg_begin;
  const int64_t item = (local >> 6) * 8 + (local & 7);
  if (item >= ws.count) return;
  const AnterpItem<TC, TP>& it = ((const AnterpItem<TC, TP>*)ws.items)[item];
  const int z0 = (int)((local >> 3) & 7) * SL;
  const gview<const double> __restrict__ W = gl(ws.w);
  const int tid = threadIdx.x;
  for (int i = tid; i < 2 * NB * NB; i += NB * NB) {
    const int cc = i / (NB * NB), r = (i / NB) % NB, m = i % NB;
    w[cc][r][m] = T(W[(cc * NB + r) * NB + m]);
  }
  const int a = tid % NB, b = tid / NB;          // (X, Y) in the z pass; (x or X, y) later
  int gmask = 0;                                 // (cx, cy) groups with a child
  T zs[4][SL];
#pragma unroll
  for (int g = 0; g < 4; ++g)
#pragma unroll
    for (int zz = 0; zz < SL; ++zz) zs[g][zz] = T(0);
#pragma unroll
  for (int oc = 0; oc < 8; ++oc) {                               // z: sum over cz
    const TC* ch = child_ptr<TC>(it.child[oc], it.child_in[oc], ws.in);
    if (!ch) continue;
    const int g = oc & 3, cz = oc >> 2;
    gmask |= 1 << g;
    T v[NB];
#pragma unroll
    for (int Z = 0; Z < NB; ++Z) v[Z] = T(gl(ch)[(Z * NB + b) * NB + a]);
#pragma unroll
    for (int zz = 0; zz < SL; ++zz)
#pragma unroll
      for (int Z = 0; Z < NB; ++Z) zs[g][zz] += T(W[(cz * NB + Z) * NB + z0 + zz]) * v[Z];
  }
#pragma unroll
  for (int g = 0; g < 4; ++g)
#pragma unroll
    for (int zz = 0; zz < SL; ++zz) t1[g][zz][b][a] = zs[g][zz];
  __syncthreads();
  // y and x passes: a thread's output (a, b) is fixed, so the weight columns w[c][.][b] and
  // w[c][.][a] it needs are read into registers once
  {
    T wy[2][NB];
#pragma unroll
    for (int cy = 0; cy < 2; ++cy)
#pragma unroll
      for (int Y = 0; Y < NB; ++Y) wy[cy][Y] = w[cy][Y][b];
#pragma unroll
    for (int cx = 0; cx < 2; ++cx)                               // y: sum over cy
#pragma unroll
      for (int zz = 0; zz < SL; ++zz) {
        T s = 0;
#pragma unroll
        for (int cy = 0; cy < 2; ++cy) {
          if (!((gmask >> (cx + 2 * cy)) & 1)) continue;
#pragma unroll
          for (int Y = 0; Y < NB; ++Y) s += wy[cy][Y] * t1[cx + 2 * cy][zz][Y][a];
        }
        t2[cx][zz][b][a] = s;
      }
  }
  __syncthreads();
  T acc[SL];
  {
    T wx[2][NB];
#pragma unroll
    for (int cx = 0; cx < 2; ++cx)
#pragma unroll
      for (int X = 0; X < NB; ++X) wx[cx][X] = w[cx][X][a];
#pragma unroll
    for (int zz = 0; zz < SL; ++zz) {                            // x: sum over cx
      T s = 0;
#pragma unroll
      for (int cx = 0; cx < 2; ++cx) {
        if (!((gmask >> cx) & 5)) continue;
#pragma unroll
        for (int X = 0; X < NB; ++X) s += wx[cx][X] * t2[cx][zz][b][X];
      }
      acc[zz] = s;
    }
  }
  const gview<TP> dst = gl(it.dst);
#pragma unroll
  for (int zz = 0; zz < SL; ++zz) dst[((z0 + zz) * NB + b) * NB + a] = acc[zz];
}

// The combine and the convert stream a few bytes per cell: each block is split over
// split_of<NB>() workgroups (a quarter of its cells each on 16^3 blocks), so that a level's
// launch has enough wavefronts in flight to cover the memory latency.
template <int NB> constexpr int split_of() { return per_thread<NB>() >= 4 ? 4 : per_thread<NB>(); }

template <int NB, typename T>
__global__ __launch_bounds__(kOpThreads) void combine_kernel(SetTable sets) {
  constexpr int N3 = NB * NB * NB, SP = split_of<NB>();
  const int set = find_set(sets, blockIdx.x);
  const WorkSet& ws = sets.s[set];
  const int64_t local = blockIdx.x - ws.wg_begin;
  const CombineItem<T>& it = ((const CombineItem<T>*)ws.items)[local / SP];
  const int c0 = (int)(local % SP) * (N3 / SP);         // this workgroup's cells c0 .. + N3 / SP
  const double sc = it.scale;
  const gview<double> dd = gl(it.dst_d ? it.dst_d : ws.out + it.dst_out) + c0;
  constexpr int PT = per_thread<NB>() / SP;
  double v[PT];
#pragma unroll
  for (int j = 0; j < PT; ++j) v[j] = it.v ? double(gl(it.v + c0)[threadIdx.x + j * kOpThreads]) : 0.0;
  if (it.far) {
#pragma unroll
    for (int j = 0; j < PT; ++j) v[j] += double(gl(it.far + c0)[threadIdx.x + j * kOpThreads]);
  }
#pragma unroll
  for (int j = 0; j < PT; ++j) v[j] *= sc;
  if (it.base) {
#pragma unroll
    for (int j = 0; j < PT; ++j) v[j] += gl(it.base + c0)[threadIdx.x + j * kOpThreads];
  }
  if (!it.dst_d && (ws.aux & kAuxAccumulate)) {       // defect-correction update of u
#pragma unroll
    for (int j = 0; j < PT; ++j) v[j] += dd[threadIdx.x + j * kOpThreads];
  }
#pragma unroll
  for (int j = 0; j < PT; ++j) dd[threadIdx.x + j * kOpThreads] = v[j];
}

template <int NB, typename T>
__global__ __launch_bounds__(kOpThreads) void convert_kernel(SetTable sets) {
  constexpr int N3 = NB * NB * NB, SP = split_of<NB>();
  const int set = find_set(sets, blockIdx.x);
  const WorkSet& ws = sets.s[set];
  const int64_t local = blockIdx.x - ws.wg_begin;
  const ConvertItem<T>& it = ((const ConvertItem<T>*)ws.items)[local / SP];
  const int c0 = (int)(local % SP) * (N3 / SP);
  const gview<const double> src = gl(it.src ? it.src : ws.in + it.src_in) + c0;
  constexpr int PT = per_thread<NB>() / SP;
  double v[PT];
#pragma unroll
  for (int j = 0; j < PT; ++j) v[j] = src[threadIdx.x + j * kOpThreads];
  const gview<T> dst = gl(it.dst) + c0;
#pragma unroll
  for (int j = 0; j < PT; ++j) dst[threadIdx.x + j * kOpThreads] = T(v[j]);
}

template <int NB>
__global__ __launch_bounds__(kOpThreads) void coarsen_kernel(SetTable sets) {
  constexpr int N3 = NB * NB * NB, HB = NB / 2;
  const int set = find_set(sets, blockIdx.x);
  const WorkSet& ws = sets.s[set];
  const CoarsenItem& it = ((const CoarsenItem*)ws.items)[blockIdx.x - ws.wg_begin];
  constexpr int PT = per_thread<NB>(), G = PT < 8 ? PT : 8;   // groups of G cells (registers)
  const gview<double> dst = gl(it.dst);
#pragma unroll 1
  for (int j0 = 0; j0 < PT; j0 += G) {
    double out[G];
#pragma unroll
    for (int jj = 0; jj < G; ++jj) {
      const int j = jj, i = threadIdx.x + (j0 + jj) * kOpThreads;
      const int x = i % NB, y = (i / NB) % NB, z = i / (NB * NB);
      const int oc = (x / HB) + 2 * (y / HB) + 4 * (z / HB);
      const gview<const double> ch = gl(it.child[oc] ? it.child[oc] : ws.in + it.child_in[oc]);
      const int fx = 2 * (x % HB), fy = 2 * (y % HB), fz = 2 * (z % HB);
      double s = 0.0;
#pragma unroll
      for (int dz = 0; dz < 2; ++dz)
#pragma unroll
        for (int dy = 0; dy < 2; ++dy)
#pragma unroll
          for (int dx = 0; dx < 2; ++dx) s += ch[((fz + dz) * NB + fy + dy) * NB + fx + dx];
      out[j] = 0.125 * s;
    }
#pragma unroll
    for (int jj = 0; jj < G; ++jj) dst[threadIdx.x + (j0 + jj) * kOpThreads] = out[jj];
  }
}

// Quadratic refinement table: row j in [-1, 2 NB] at index j + 1 holds {lo, w0, w1, w2}.
template <int NB, typename T>
__device__ __forceinline__ T refine_point(gview<const T> __restrict__ pw,
                                          gview<const double> __restrict__ w3, int jx, int jy, int jz) {
  const gview<const double> rx = w3 + 4 * (jx + 1);
  const gview<const double> ry = w3 + 4 * (jy + 1);
  const gview<const double> rz = w3 + 4 * (jz + 1);
  const int lx = (int)rx[0], ly = (int)ry[0], lz = (int)rz[0];
  T s = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    T sy = 0;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const gview<const T> row = pw + ((lz + a) * NB + (ly + b)) * NB + lx;
      const T sx = T(rx[1]) * row[0] + T(rx[2]) * row[1] + T(rx[3]) * row[2];
      sy += T(ry[1 + b]) * sx;
    }
    s += T(rz[1 + a]) * sy;
  }
  return s;
}

// Jw on a child block: the quadratic is separable, so it is applied along x, then y, then z
// through LDS over the parent cells the octant's stencils touch (R = NB/2 + 2 per axis, from
// the first child cell's stencil start; the planner checks that every stencil of the octant
// lies inside that range).
template <int NB>
__global__ __launch_bounds__(kOpThreads) void refine_kernel(SetTable sets) {
  constexpr int R = NB / 2 + 2, PT = per_thread<NB>();
  constexpr int R3 = R * R * R, PL = R3 > R * NB * NB ? R3 : R * NB * NB;
  __shared__ double pl[PL];              // parent region [z][y][x], then the y pass [z][y][X]
  __shared__ double t1[R * R * NB];      // x pass [z][y][X]
  __shared__ double tab[3][NB][4];       // per axis and child index: stencil start - base, w0..w2
  const int set = find_set(sets, blockIdx.x);
  const WorkSet& ws = sets.s[set];
  const RefineItem& it = ((const RefineItem*)ws.items)[blockIdx.x - ws.wg_begin];
  const gview<const double> __restrict__ w3 = gl(ws.w);
  const gview<const double> __restrict__ pw = gl(it.parent_w);
  const int c[3] = {it.octant & 1, (it.octant >> 1) & 1, (it.octant >> 2) & 1};
  // table row of child index j along axis d: w3[4 (c_d NB + j + 1) ...]
  const int b0 = (int)w3[4 * (c[0] * NB + 1)], b1 = (int)w3[4 * (c[1] * NB + 1)],
            b2 = (int)w3[4 * (c[2] * NB + 1)];
  if (threadIdx.x < 3 * NB) {
    const int d = threadIdx.x / NB, j = threadIdx.x % NB;
    const gview<const double> r = w3 + 4 * (c[d] * NB + j + 1);
    const int base = d == 0 ? b0 : d == 1 ? b1 : b2;
    tab[d][j][0] = r[0] - base;
    tab[d][j][1] = r[1];
    tab[d][j][2] = r[2];
    tab[d][j][3] = r[3];
  }
  {
    constexpr int RP = (R3 + kOpThreads - 1) / kOpThreads;
    double v[RP];
#pragma unroll
    for (int h = 0; h < RP; ++h) {
      const int i = threadIdx.x + h * kOpThreads;
      const int x = b0 + i % R, y = b1 + (i / R) % R, z = b2 + i / (R * R);
      v[h] = (i < R3 && x < NB && y < NB && z < NB) ? pw[(z * NB + y) * NB + x] : 0.0;
    }
#pragma unroll
    for (int h = 0; h < RP; ++h)
      if (threadIdx.x + h * kOpThreads < R3) pl[threadIdx.x + h * kOpThreads] = v[h];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < R * R * NB; i += kOpThreads) {        // x
    const int X = i % NB, zy = i / NB;
    const int lo = (int)tab[0][X][0];
    const double* row = pl + zy * R + lo;
    t1[i] = tab[0][X][1] * row[0] + tab[0][X][2] * row[1] + tab[0][X][3] * row[2];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < R * NB * NB; i += kOpThreads) {       // y
    const int X = i % NB, Y = (i / NB) % NB, z = i / (NB * NB);
    const int lo = (int)tab[1][Y][0];
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) s += tab[1][Y][1 + k] * t1[(z * R + lo + k) * NB + X];
    pl[i] = s;
  }
  __syncthreads();
  double out[PT];
#pragma unroll
  for (int j = 0; j < PT; ++j) {                                       // z
    const int i = threadIdx.x + j * kOpThreads;
    const int XY = i % (NB * NB), Z = i / (NB * NB);
    const int lo = (int)tab[2][Z][0];
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) s += tab[2][Z][1 + k] * pl[(lo + k) * NB * NB + XY];
    out[j] = s;
  }
  const gview<double> jw = gl(it.jw);
#pragma unroll
  for (int j = 0; j < PT; ++j) jw[threadIdx.x + j * kOpThreads] = out[j];
}

// g = f - h^-2 L(Jw): the block's Jw and its one-cell halo are staged in LDS; a halo cell is the
// face-adjacent neighbour block's Jw where that block exists, else the parent's quadratic
// extended one child cell outward (each halo cell computed by one thread).
template <int NB, typename T>
__global__ __launch_bounds__(kOpThreads) void correct_kernel(SetTable sets) {
  constexpr int E = NB + 2, PT = per_thread<NB>();
  __shared__ double ext[E * E * E];
  const int set = find_set(sets, blockIdx.x);
  const WorkSet& ws = sets.s[set];
  const CorrectItem<T>& it = ((const CorrectItem<T>*)ws.items)[blockIdx.x - ws.wg_begin];
  const gview<const double> __restrict__ w3 = gl(ws.w);
  const gview<const double> __restrict__ f = gl(it.f ? it.f : ws.in + it.f_in);
  const gview<const double> __restrict__ jw = gl(it.jw);
  const gview<const double> __restrict__ pw = gl(it.parent_w);
  const int c[3] = {it.octant & 1, (it.octant >> 1) & 1, (it.octant >> 2) & 1};
  double fv[PT], jv[PT];
#pragma unroll
  for (int j = 0; j < PT; ++j) fv[j] = f[threadIdx.x + j * kOpThreads];
#pragma unroll
  for (int j = 0; j < PT; ++j) jv[j] = jw[threadIdx.x + j * kOpThreads];
  // halo cells (6 NB^2) spread over the threads
  constexpr int HP = (6 * NB * NB + kOpThreads - 1) / kOpThreads;
#pragma unroll 1
  for (int h = 0; h < HP; ++h) {
    const int jj = threadIdx.x + h * kOpThreads;
    if (jj >= 6 * NB * NB) break;
    const int face = jj / (NB * NB), j = jj % (NB * NB);
    const int ax = face >> 1, hi = face & 1;
    const int a = j % NB, b = j / NB;
    int q[3];                              // halo cell in the block's coordinates (-1 or NB on ax)
    const int o = hi ? NB : -1;
    if (ax == 0) { q[0] = o; q[1] = a; q[2] = b; }
    else if (ax == 1) { q[0] = a; q[1] = o; q[2] = b; }
    else { q[0] = a; q[1] = b; q[2] = o; }
    double v;
    if (const double* nb = it.nbr[face]) {
      int p[3] = {q[0], q[1], q[2]};
      p[ax] = hi ? 0 : NB - 1;
      v = gl(nb)[(p[2] * NB + p[1]) * NB + p[0]];
    } else {
      v = refine_point<NB, double>(pw, w3, c[0] * NB + q[0], c[1] * NB + q[1], c[2] * NB + q[2]);
    }
    ext[((q[2] + 1) * E + q[1] + 1) * E + q[0] + 1] = v;
  }
#pragma unroll
  for (int j = 0; j < PT; ++j) {
    const int i = threadIdx.x + j * kOpThreads;
    const int x = i % NB, y = (i / NB) % NB, z = i / (NB * NB);
    ext[((z + 1) * E + y + 1) * E + x + 1] = jv[j];
  }
  __syncthreads();
  const double inv_h2 = it.inv_h2;
  T out[PT];
#pragma unroll
  for (int j = 0; j < PT; ++j) {
    const int i = threadIdx.x + j * kOpThreads;
    const int x = i % NB, y = (i / NB) % NB, z = i / (NB * NB);
    const int cc = ((z + 1) * E + y + 1) * E + x + 1;
    const double lap = ext[cc - 1] + ext[cc + 1] + ext[cc - E] + ext[cc + E] + ext[cc - E * E] +
                       ext[cc + E * E] - 6.0 * ext[cc];
    out[j] = T(fv[j] - inv_h2 * lap);
  }
  const gview<T> g = gl(it.g);
#pragma unroll
  for (int j = 0; j < PT; ++j) g[threadIdx.x + j * kOpThreads] = out[j];
}

// r = f - h^-2 (sum of 6 neighbours - 6 u) on cells whose neighbours all exist.  One workgroup
// per (block, z-slab of NB / kResidualSlabs planes) and one thread per (x, y) column: the slab
// and its one-cell halo (from the block itself or the face-adjacent same-level blocks) are
// staged in LDS.  Writes r in FP64 and/or its FP32 rounding (null pointers skip).
template <int NB>
__global__ __launch_bounds__(NB * NB) void residual_kernel(SetTable sets) {
  constexpr int SZ = NB / kResidualSlabs, E = NB + 2, N2 = NB * NB;
  __shared__ double ext[(SZ + 2) * E * E];
  const int set = find_set(sets, blockIdx.x);
  const WorkSet& ws = sets.s[set];
  // XCD x (workgroup w runs on XCD w mod 8; set starts are multiples of 8) takes the items
  // [x nper, (x + 1) nper): neighbour blocks, mostly nearby in layout order, share its L2
  const int64_t local = blockIdx.x - ws.wg_begin;
  const int64_t nper = (ws.count + 7) / 8, jw = local >> 3;
  const int64_t item = (local & 7) * nper + jw / kResidualSlabs;
  if (item >= ws.count) return;
  const ResidualItem& it = ((const ResidualItem*)ws.items)[item];
  const int z0 = (int)(jw % kResidualSlabs) * SZ;
  const gview<double> r = gl(it.r);
  const gview<float> conv = gl(it.conv);
  if (!r && !conv) return;
  const int t = threadIdx.x, x = t % NB, y = t / NB;
  if (!it.leaf) {
#pragma unroll
    for (int j = 0; j < SZ; ++j) {
      const int i = (z0 + j) * N2 + t;
      if (r) r[i] = 0.0;
      if (conv) conv[i] = 0.0f;
    }
    return;
  }
  const gview<const double> __restrict__ f = gl(ws.in + it.off);
  const gview<const double> __restrict__ u = gl(ws.out + it.off);
  const gview<const double> out_all = gl((const double*)ws.out);
  int missing = 0;
#pragma unroll
  for (int face = 0; face < 6; ++face)
    if (it.nbr_off[face] < 0) missing |= 1 << face;
  // own planes z0 - 1 .. z0 + SZ (the outer two from the z neighbours at the block faces)
  double fv[SZ], uv[SZ + 2];
#pragma unroll
  for (int j = 0; j < SZ; ++j) fv[j] = f[(z0 + j) * N2 + t];
#pragma unroll
  for (int j = 0; j < SZ + 2; ++j) {
    const int z = z0 - 1 + j;
    uv[j] = 0.0;
    if (z >= 0 && z < NB) uv[j] = u[z * N2 + t];
    else if (z < 0 && !(missing & 16)) uv[j] = out_all[it.nbr_off[4] + (NB - 1) * N2 + t];
    else if (z >= NB && !(missing & 32)) uv[j] = out_all[it.nbr_off[5] + t];
  }
  // x and y faces of the slab's planes: 4 faces x NB x SZ cells over the threads
  constexpr int HP = (4 * NB * SZ + N2 - 1) / N2;
  double hv[HP];
  int hq[HP];
#pragma unroll
  for (int h = 0; h < HP; ++h) {
    const int jj = t + h * N2;
    hq[h] = -1;
    if (jj >= 4 * NB * SZ) continue;
    const int face = jj / (NB * SZ), rem = jj % (NB * SZ), a = rem % NB, zz = rem / NB;
    if ((missing >> face) & 1) continue;
    const gview<const double> nb = out_all + it.nbr_off[face];
    const int ax = face >> 1, hi = face & 1;
    const int src = hi ? 0 : NB - 1, dst = hi ? NB + 1 : 0;
    int px, py, qx, qy;                   // cell in the neighbour, halo cell in ext
    if (ax == 0) { px = src; py = a; qx = dst; qy = a + 1; }
    else { px = a; py = src; qx = a + 1; qy = dst; }
    hq[h] = ((zz + 1) * E + qy) * E + qx;
    hv[h] = nb[(z0 + zz) * N2 + py * NB + px];
  }
#pragma unroll
  for (int j = 0; j < SZ + 2; ++j) ext[(j * E + y + 1) * E + x + 1] = uv[j];
#pragma unroll
  for (int h = 0; h < HP; ++h)
    if (hq[h] >= 0) ext[hq[h]] = hv[h];
  __syncthreads();
  const double inv_h2 = it.inv_h2;
  double out[SZ];
#pragma unroll
  for (int j = 0; j < SZ; ++j) {
    const int z = z0 + j;
    const bool edge = ((missing & 1) && x == 0) || ((missing & 2) && x == NB - 1) ||
                      ((missing & 4) && y == 0) || ((missing & 8) && y == NB - 1) ||
                      ((missing & 16) && z == 0) || ((missing & 32) && z == NB - 1);
    const int c = ((j + 1) * E + y + 1) * E + x + 1;
    const double lap = ext[c - 1] + ext[c + 1] + ext[c - E] + ext[c + E] + ext[c - E * E] +
                       ext[c + E * E] - 6.0 * ext[c];
    out[j] = edge ? 0.0 : fv[j] - inv_h2 * lap;
  }
#pragma unroll
  for (int j = 0; j < SZ; ++j) {
    const int i = (z0 + j) * N2 + t;
    if (r) r[i] = out[j];
    if (conv) conv[i] = float(out[j]);
  }
}

}  // namespace

#define LGF_NB_DISPATCH(nb, ...)                                           \
  do {                                                                     \
    if ((nb) == 16) { constexpr int NB = 16; __VA_ARGS__; }                \
    else if ((nb) == 8) { constexpr int NB = 8; __VA_ARGS__; }             \
    else return hipErrorInvalidValue;                                      \
  } while (0)

#define LGF_LAUNCH_SIMPLE(...)                                                   \
  const int64_t wg = assign_wg(t, 1);                                             \
  if (wg == 0) return hipSuccess;                                                 \
  LGF_NB_DISPATCH(nb, __VA_ARGS__<<<(unsigned)wg, kOpThreads, 0, st>>>(t));       \
  return hipGetLastError();

template <typename TC, typename TP> hipError_t launch_anterp(int nb, SetTable& t, hipStream_t st) {
  int64_t wg = 0;                                // 64 workgroups per 8 parents (see anterp_kernel)
  for (int i = 0; i < t.n; ++i) {
    t.s[i].wg_begin = wg;
    wg += (t.s[i].count + 7) / 8 * 64;
  }
  if (wg == 0) return hipSuccess;
  LGF_NB_DISPATCH(nb, anterp_kernel<NB, TC, TP><<<(unsigned)wg, NB * NB, 0, st>>>(t));
  return hipGetLastError();
}
template <typename TC, typename TP> hipError_t launch_interp(int nb, SetTable& t, hipStream_t st) {
  LGF_LAUNCH_SIMPLE(interp_kernel<NB, TC, TP>)
}
template <typename T> hipError_t launch_combine(int nb, SetTable& t, hipStream_t st) {
  const int64_t wg = assign_wg(t, nb == 16 ? split_of<16>() : split_of<8>());
  if (wg == 0) return hipSuccess;
  LGF_NB_DISPATCH(nb, combine_kernel<NB, T><<<(unsigned)wg, kOpThreads, 0, st>>>(t));
  return hipGetLastError();
}
template <typename T> hipError_t launch_convert(int nb, SetTable& t, hipStream_t st) {
  const int64_t wg = assign_wg(t, nb == 16 ? split_of<16>() : split_of<8>());
  if (wg == 0) return hipSuccess;
  LGF_NB_DISPATCH(nb, convert_kernel<NB, T><<<(unsigned)wg, kOpThreads, 0, st>>>(t));
  return hipGetLastError();
}
hipError_t launch_coarsen(int nb, SetTable& t, hipStream_t st) {
  LGF_LAUNCH_SIMPLE(coarsen_kernel<NB>)
}
hipError_t launch_refine(int nb, SetTable& t, hipStream_t st) {
  LGF_LAUNCH_SIMPLE(refine_kernel<NB>)
}
template <typename T> hipError_t launch_correct(int nb, SetTable& t, hipStream_t st) {
  LGF_LAUNCH_SIMPLE(correct_kernel<NB, T>)
}
hipError_t launch_residual(int nb, SetTable& t, hipStream_t st) {
  int64_t wg = 0;                                // 8 ceil(count / 8) blocks of slabs per set
  for (int i = 0; i < t.n; ++i) {
    t.s[i].wg_begin = wg;
    wg += (t.s[i].count + 7) / 8 * 8 * kResidualSlabs;
  }
  if (wg == 0) return hipSuccess;
  LGF_NB_DISPATCH(nb, residual_kernel<NB><<<(unsigned)wg, NB * NB, 0, st>>>(t));
  return hipGetLastError();
}

// Forward operators of the per-level lattice (Sec. 3: applications need at least the gradient of
// the computed field; the source correction makes each level's 7-point operator consistent with
// the computed inverse).  Laplacian h^-2 (6 neighbours - 6 centre); gradient by central
// differences (u(x + e_a) - u(x - e_a)) / 2h; curl of a three-component field from the same
// differences.  A neighbour across a block face comes from the same-level block on that side;
// where there is none, from the block's parent field, the parent's quadratic extended one child
// cell outward (the ghost of the source correction), or, on the coarsest level, nowhere: those
// cells, and every cell of a non-leaf block, are 0.  One workgroup per (block, z-slab of
// NB / kResidualSlabs planes), one thread per (x, y) column: each input component's slab and its
// one-cell halo are staged in LDS (each halo cell computed once), then every output of the slab
// is formed from LDS and stored coalesced.
// workgroups (z-slabs) per block of the forward operators: 2 for one input component, 4 for
// three (their LDS slabs would hold the occupancy down)
template <int NIN> constexpr int op_slabs() { return NIN == 1 ? 2 : 4; }

template <int NB, int NIN>
__global__ __launch_bounds__(NB * NB) void fwd_op_kernel(const OpItem* __restrict__ items, int64_t nblk, int op,
                                                         const double* __restrict__ u, double* __restrict__ out,
                                                         int64_t cs, const double* __restrict__ w3tab) {
  constexpr int SLABS = op_slabs<NIN>();
  constexpr int SZ = NB / SLABS, E = NB + 2, N2 = NB * NB, PL = E * E, SL = (SZ + 2) * PL;
  constexpr int NH = 4 * NB * SZ;           // x and y halo cells of the slab's planes
  __shared__ double ext[NIN * SL];
  // workgroup w runs on XCD w mod 8; XCD x takes the blocks [x nper, (x + 1) nper) of the
  // layout, so that the halo cells a block reads from its neighbours (in layout order mostly
  // nearby) are in that XCD's L2
  const int64_t nper = (nblk + 7) / 8, j = blockIdx.x >> 3;
  const int64_t blk = (blockIdx.x & 7) * nper + j / SLABS;
  if (blk >= nblk) return;
  const OpItem& it = items[blk];
  const int z0 = (int)(j % SLABS) * SZ;
  const int t = threadIdx.x, x = t % NB, y = t / NB;
  const int nout = op == 0 ? 1 : 3;
  const gview<double> o = gl(out);
  if (!it.leaf) {
    for (int c = 0; c < nout; ++c)
#pragma unroll
      for (int j = 0; j < SZ; ++j) o[c * cs + it.off + (z0 + j) * N2 + t] = 0.0;
    return;
  }
  const gview<const double> U = gl(u);
  const gview<const double> w3 = gl(w3tab);
  const int oc[3] = {it.octant & 1, (it.octant >> 1) & 1, (it.octant >> 2) & 1};
  const bool ghost = it.par_off >= 0;
  // component c at cell q of the block's frame; at most one coordinate is -1 or NB
  auto cell = [&](int c, int qx, int qy, int qz) -> double {
    const int64_t cb = (int64_t)c * cs;
    int face = -1, q[3] = {qx, qy, qz};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (q[a] < 0) face = 2 * a;
      else if (q[a] >= NB) face = 2 * a + 1;
    }
    if (face < 0) return U[cb + it.off + (qz * NB + qy) * NB + qx];
    const int64_t nb = it.nbr_off[face];
    if (nb >= 0) {
      const int a = face >> 1;
      q[a] = (face & 1) ? 0 : NB - 1;
      return U[cb + nb + (q[2] * NB + q[1]) * NB + q[0]];
    }
    if (ghost) return refine_point<NB, double>(U + cb + it.par_off, w3, oc[0] * NB + qx, oc[1] * NB + qy, oc[2] * NB + qz);
    return 0.0;
  };
  // the own column (all loads issued before the LDS stores; the slab's own cells directly, only
  // the two z-halo cells through cell()), then the x and y halo cells
#pragma unroll
  for (int c = 0; c < NIN; ++c) {
    double col[SZ + 2];
    const gview<const double> Uc = U + (int64_t)c * cs + it.off + (z0 * NB + y) * NB + x;
#pragma unroll
    for (int j = 0; j < SZ; ++j) col[j + 1] = Uc[j * N2];
    col[0] = cell(c, x, y, z0 - 1);
    col[SZ + 1] = cell(c, x, y, z0 + SZ);
#pragma unroll
    for (int j = 0; j < SZ + 2; ++j) ext[c * SL + j * PL + (y + 1) * E + x + 1] = col[j];
  }
  for (int hc = t; hc < NH; hc += N2) {
    const int hf = hc / (NB * SZ), hr = hc % (NB * SZ), ha = hr % NB, hz = hr / NB;
    const int qx = hf == 0 ? -1 : hf == 1 ? NB : ha, qy = hf == 2 ? -1 : hf == 3 ? NB : ha;
#pragma unroll
    for (int c = 0; c < NIN; ++c) ext[c * SL + (hz + 1) * PL + (qy + 1) * E + qx + 1] = cell(c, qx, qy, z0 + hz);
  }
  __syncthreads();
  const double ih = it.inv_h, hh = 0.5 * it.inv_h;
#pragma unroll
  for (int j = 0; j < SZ; ++j) {
    const int z = z0 + j;
    bool ok = true;
    if (!ghost) {
      ok = !((x == 0 && it.nbr_off[0] < 0) || (x == NB - 1 && it.nbr_off[1] < 0) ||
             (y == 0 && it.nbr_off[2] < 0) || (y == NB - 1 && it.nbr_off[3] < 0) ||
             (z == 0 && it.nbr_off[4] < 0) || (z == NB - 1 && it.nbr_off[5] < 0));
    }
    const int cc = (j + 1) * PL + (y + 1) * E + x + 1;
    const int64_t at = it.off + (int64_t)z * N2 + t;
    auto d = [&](int c, int step) { return (ext[c * SL + cc + step] - ext[c * SL + cc - step]) * hh; };
    if (op == 0) {
      const double lap = ext[cc - 1] + ext[cc + 1] + ext[cc - E] + ext[cc + E] + ext[cc - PL] + ext[cc + PL] -
                         6.0 * ext[cc];
      o[at] = ok ? ih * ih * lap : 0.0;
    } else if (op == 1) {
      o[at] = ok ? d(0, 1) : 0.0;
      o[cs + at] = ok ? d(0, E) : 0.0;
      o[2 * cs + at] = ok ? d(0, PL) : 0.0;
    } else if constexpr (NIN == 3) {
      o[at] = ok ? d(2, E) - d(1, PL) : 0.0;
      o[cs + at] = ok ? d(0, PL) - d(2, 1) : 0.0;
      o[2 * cs + at] = ok ? d(1, 1) - d(0, E) : 0.0;
    }
  }
}

hipError_t launch_fwd_op(int nb, int op, const OpItem* items, int64_t n, const double* u, double* out,
                         const double* w3, hipStream_t st) {
  if (n == 0) return hipSuccess;
  if (!items || !w3 || op < 0 || op > 2) return hipErrorInvalidValue;
  const int64_t n3 = (int64_t)nb * nb * nb;
  const int64_t nper = (n + 7) / 8;             // blocks per XCD (see fwd_op_kernel)
  if (op == 2) {
    const unsigned g = (unsigned)(8 * nper * op_slabs<3>());
    LGF_NB_DISPATCH(nb, (fwd_op_kernel<NB, 3><<<g, NB * NB, 0, st>>>(items, n, op, u, out, n * n3, w3)));
  } else {
    const unsigned g = (unsigned)(8 * nper * op_slabs<1>());
    LGF_NB_DISPATCH(nb, (fwd_op_kernel<NB, 1><<<g, NB * NB, 0, st>>>(items, n, op, u, out, n * n3, w3)));
  }
  return hipGetLastError();
}

template hipError_t launch_anterp<float, float>(int, SetTable&, hipStream_t);
template hipError_t launch_anterp<double, double>(int, SetTable&, hipStream_t);
template hipError_t launch_anterp<float, double>(int, SetTable&, hipStream_t);
template hipError_t launch_interp<float, float>(int, SetTable&, hipStream_t);
template hipError_t launch_interp<double, double>(int, SetTable&, hipStream_t);
template hipError_t launch_interp<float, double>(int, SetTable&, hipStream_t);

#define LGF_INST(T)                                                       \
  template hipError_t launch_combine<T>(int, SetTable&, hipStream_t);     \
  template hipError_t launch_convert<T>(int, SetTable&, hipStream_t);     \
  template hipError_t launch_correct<T>(int, SetTable&, hipStream_t);
LGF_INST(float)
LGF_INST(double)

}  // namespace lgf
