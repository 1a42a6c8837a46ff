// Refinement-criterion layout builder on the GPU (Sec. 3, Convergence subsection, eq. ref_crit).
//
// One adaptation step of a block layout from a field on its cells (the vorticity of a flow, or
// the source of a Poisson problem): omega of a block is its largest |value|, omega_max of level l
// the largest over the level; a level-l block is flagged when omega > alpha^(L_R - 1 - l)
// omega_max and l < L_R - 1 (the exponent and the strict comparison are this library's reading).
// The new layout keeps the base level; its level-(l+1) blocks are the 8 children of the flagged
// level-l blocks, and only blocks of the old layout (where the field is known) can be flagged.
// Order of the new layout: base blocks in their old order, then per level the children of each
// flagged block in the new order of the flagged blocks, child offset (cx, cy, cz) with cz
// fastest.  Repeating the step from the base layout with the field evaluated on each new layout
// builds a layout with L_R levels one level at a time.
//
// Kernels: block |max| (one workgroup per block, the only pass over the field), per-level
// maxima and thresholds (one workgroup), an open-addressing hash of the old layout's
// (level, x, y, z) keys, and per new level: flags, an exclusive scan (one workgroup) and the
// emission of children with the lookup of each child in the old layout.
#include <vector>

#include "kernels.hpp"

namespace lgf {

namespace {

constexpr int kMaxLevels = 16;
constexpr uint64_t kEmpty = ~0ull;

__device__ __forceinline__ uint64_t block_key(int l, int x, int y, int z) {
  // 4 bits of level, 20 bits per coordinate (offset so that negative coordinates fit)
  const uint64_t o = 1u << 19;
  return ((uint64_t)l << 60) | (((uint64_t)(x + o) & 0xFFFFF) << 40) | (((uint64_t)(y + o) & 0xFFFFF) << 20) |
         ((uint64_t)(z + o) & 0xFFFFF);
}

__device__ __forceinline__ uint32_t key_hash(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return (uint32_t)k;
}

template <int NB>
__global__ __launch_bounds__(256) void block_absmax_kernel(const double* __restrict__ f, double* __restrict__ omega) {
  constexpr int N3 = NB * NB * NB;
  __shared__ double red[4];
  const gview<const double> src = gl(f + (int64_t)blockIdx.x * N3);
  double m = 0.0;
  for (int c = threadIdx.x; c < N3; c += 256) m = fmax(m, fabs(src[c]));
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) gl(omega)[blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// per level: omega_max and the threshold alpha^(L_R - 1 - l) omega_max (alpha^k by repeated
// multiplication); one workgroup of 1024 threads
__global__ __launch_bounds__(1024) void thresholds_kernel(const int32_t* __restrict__ levels,
                                                          const double* __restrict__ omega, int64_t n,
                                                          int n_levels, double alpha, double* __restrict__ thr,
                                                          int32_t* __restrict__ bad) {
  __shared__ double lm[kMaxLevels][16];
  double mine[kMaxLevels];
#pragma unroll
  for (int l = 0; l < kMaxLevels; ++l) mine[l] = -1.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) {
    const int l = levels[i];
    if (l < 0 || l >= kMaxLevels) {
      gl(bad)[0] = 1;
      continue;
    }
#pragma unroll
    for (int q = 0; q < kMaxLevels; ++q)
      if (q == l) mine[q] = fmax(mine[q], omega[i]);
  }
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int l = 0; l < kMaxLevels; ++l) {
    double m = mine[l];
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) lm[l][w] = m;
  }
  __syncthreads();
  if (threadIdx.x < kMaxLevels) {
    const int l = threadIdx.x;
    double m = -1.0;
    for (int q = 0; q < 16; ++q) m = fmax(m, lm[l][q]);
    double a = 1.0;
    for (int k = 0; k < n_levels - 1 - l; ++k) a *= alpha;
    gl(thr)[l] = m < 0.0 ? -1.0 : a * m;            // -1: the level has no blocks
  }
}

__global__ __launch_bounds__(256) void hash_insert_kernel(const int32_t* __restrict__ blocks,
                                                          const int32_t* __restrict__ levels, int64_t n,
                                                          unsigned long long* keys, int32_t* vals, uint32_t mask,
                                                          int32_t* bad) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const uint64_t k = block_key(levels[i], blocks[3 * i], blocks[3 * i + 1], blocks[3 * i + 2]);
  uint32_t h = key_hash(k) & mask;
  for (uint32_t probe = 0; probe <= mask; ++probe) {
    const unsigned long long prev = atomicCAS(keys + h, (unsigned long long)kEmpty, (unsigned long long)k);
    if (prev == kEmpty) {
      gl(vals)[h] = (int32_t)i;
      return;
    }
    if (prev == k) {                                 // a duplicate block in the layout
      gl(bad)[0] = 2;
      return;
    }
    h = (h + 1) & mask;
  }
  gl(bad)[0] = 3;
}

__device__ __forceinline__ int32_t hash_find(const unsigned long long* keys, const int32_t* vals, uint32_t mask,
                                             uint64_t k) {
  uint32_t h = key_hash(k) & mask;
  for (uint32_t probe = 0; probe <= mask; ++probe) {
    const unsigned long long v = keys[h];
    if (v == k) return vals[h];
    if (v == kEmpty) return -1;
    h = (h + 1) & mask;
  }
  return -1;
}

// base level: flags of the old layout's level-0 blocks (in old order), to be compacted
__global__ __launch_bounds__(256) void base_flags_kernel(const int32_t* __restrict__ levels, int64_t n,
                                                         int32_t* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) gl(flag)[i] = levels[i] == 0;
}

// exclusive scan of m int32 values (one workgroup of 1024); out[m] = total
__global__ __launch_bounds__(1024) void scan_kernel(const int32_t* __restrict__ in, int64_t m,
                                                    int32_t* __restrict__ out) {
  __shared__ int64_t part[1024];
  const int64_t chunk = (m + 1023) / 1024;
  const int64_t lo = std::min<int64_t>(m, threadIdx.x * chunk), hi = std::min<int64_t>(m, lo + chunk);
  int64_t s = 0;
  for (int64_t i = lo; i < hi; ++i) s += in[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int64_t v = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  int64_t run = part[threadIdx.x] - s;
  for (int64_t i = lo; i < hi; ++i) {
    const int32_t v = in[i];
    gl(out)[i] = (int32_t)run;
    run += v;
  }
  if (threadIdx.x == 1023) gl(out)[m] = (int32_t)part[1023];
}

// base level of the new layout: old level-0 block i goes to position pos[i]
__global__ __launch_bounds__(256) void emit_base_kernel(const int32_t* __restrict__ blocks,
                                                        const int32_t* __restrict__ flag,
                                                        const int32_t* __restrict__ pos, int64_t n,
                                                        int32_t* __restrict__ cur_xyz, int32_t* __restrict__ cur_old) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n || !flag[i]) return;
  const int32_t p = pos[i];
  for (int a = 0; a < 3; ++a) gl(cur_xyz)[3 * p + a] = blocks[3 * i + a];
  gl(cur_old)[p] = (int32_t)i;
}

// flags of the new layout's level-l blocks: in the old layout and meeting the criterion
__global__ __launch_bounds__(256) void level_flags_kernel(const int32_t* __restrict__ cur_old, int64_t m, int l,
                                                          int n_levels, const double* __restrict__ omega,
                                                          const double* __restrict__ thr, int32_t* __restrict__ flag) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= m) return;
  const int32_t i = cur_old[p];
  gl(flag)[p] = (i >= 0 && l < n_levels - 1 && omega[i] > thr[l]) ? 1 : 0;
}

// children of the flagged level-l blocks: level-(l+1) positions 8 rank + (cx, cy, cz) (cz
// fastest), each looked up in the old layout
__global__ __launch_bounds__(256) void emit_children_kernel(const int32_t* __restrict__ cur_xyz,
                                                            const int32_t* __restrict__ flag,
                                                            const int32_t* __restrict__ rank, int64_t m, int l,
                                                            const unsigned long long* __restrict__ keys,
                                                            const int32_t* __restrict__ vals, uint32_t mask,
                                                            int32_t* __restrict__ nxt_xyz,
                                                            int32_t* __restrict__ nxt_old) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t p = t >> 3;
  if (p >= m || !flag[p]) return;
  const int oc = (int)(t & 7);
  const int cx = oc >> 2, cy = (oc >> 1) & 1, cz = oc & 1;
  const int x = 2 * cur_xyz[3 * p] + cx, y = 2 * cur_xyz[3 * p + 1] + cy, z = 2 * cur_xyz[3 * p + 2] + cz;
  const int64_t q = 8 * (int64_t)rank[p] + oc;
  gl(nxt_xyz)[3 * q] = x;
  gl(nxt_xyz)[3 * q + 1] = y;
  gl(nxt_xyz)[3 * q + 2] = z;
  gl(nxt_old)[q] = hash_find(keys, vals, mask, block_key(l + 1, x, y, z));
}

// the level's blocks into the caller's output at offset base
__global__ __launch_bounds__(256) void copy_out_kernel(const int32_t* __restrict__ cur_xyz, int64_t m, int l,
                                                       int32_t* __restrict__ out_blocks,
                                                       int32_t* __restrict__ out_levels) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= m) return;
  for (int a = 0; a < 3; ++a) gl(out_blocks)[3 * p + a] = cur_xyz[3 * p + a];
  gl(out_levels)[p] = l;
}

unsigned grid_of(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + 255) / 256); }

struct DevBuf {
  std::vector<void*> ptrs;
  template <typename T> hipError_t get(T** p, int64_t count) {
    *p = nullptr;
    LGF_HIP_CHECK(hipMalloc((void**)p, (size_t)std::max<int64_t>(count, 1) * sizeof(T)));
    ptrs.push_back(*p);
    return hipSuccess;
  }
  ~DevBuf() {
    for (void* p : ptrs) (void)hipFree(p);
  }
};

}  // namespace

hipError_t layout_adapt(const int32_t* blocks, const int32_t* levels, int64_t n, int nb, const double* field,
                        int n_levels, double alpha, int32_t* out_blocks, int32_t* out_levels, int64_t cap,
                        int64_t* n_out, hipStream_t st) {
  if (n <= 0 || (nb != 8 && nb != 16) || n_levels < 1 || n_levels > kMaxLevels || !(alpha > 0.0))
    return hipErrorInvalidValue;
  DevBuf buf;
  double *omega = nullptr, *thr = nullptr;
  int32_t *bad = nullptr, *vals = nullptr, *flag = nullptr, *pos = nullptr;
  unsigned long long* keys = nullptr;
  uint32_t tsize = 1;
  while ((int64_t)tsize < 2 * n) tsize <<= 1;
  LGF_HIP_CHECK(buf.get(&omega, n));
  LGF_HIP_CHECK(buf.get(&thr, kMaxLevels));
  LGF_HIP_CHECK(buf.get(&bad, 1));
  LGF_HIP_CHECK(buf.get(&keys, tsize));
  LGF_HIP_CHECK(buf.get(&vals, tsize));
  LGF_HIP_CHECK(hipMemsetAsync(bad, 0, sizeof(int32_t), st));
  LGF_HIP_CHECK(hipMemsetAsync(keys, 0xFF, (size_t)tsize * sizeof(unsigned long long), st));
  if (nb == 16) block_absmax_kernel<16><<<(unsigned)n, 256, 0, st>>>(field, omega);
  else block_absmax_kernel<8><<<(unsigned)n, 256, 0, st>>>(field, omega);
  LGF_HIP_CHECK(hipGetLastError());
  thresholds_kernel<<<1, 1024, 0, st>>>(levels, omega, n, n_levels, alpha, thr, bad);
  LGF_HIP_CHECK(hipGetLastError());
  hash_insert_kernel<<<grid_of(n), 256, 0, st>>>(blocks, levels, n, keys, vals, tsize - 1, bad);
  LGF_HIP_CHECK(hipGetLastError());
  // base level of the new layout: the old level-0 blocks in order
  LGF_HIP_CHECK(buf.get(&flag, n));
  LGF_HIP_CHECK(buf.get(&pos, n + 1));
  base_flags_kernel<<<grid_of(n), 256, 0, st>>>(levels, n, flag);
  scan_kernel<<<1, 1024, 0, st>>>(flag, n, pos);
  LGF_HIP_CHECK(hipGetLastError());
  int32_t h[2] = {0, 0};
  LGF_HIP_CHECK(hipMemcpyAsync(&h[0], pos + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  LGF_HIP_CHECK(hipMemcpyAsync(&h[1], bad, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  LGF_HIP_CHECK(hipStreamSynchronize(st));
  if (h[1]) return hipErrorInvalidValue;       // level out of range or a duplicate block
  int64_t m = h[0];
  int32_t *cur_xyz = nullptr, *cur_old = nullptr;
  LGF_HIP_CHECK(buf.get(&cur_xyz, 3 * m));
  LGF_HIP_CHECK(buf.get(&cur_old, m));
  emit_base_kernel<<<grid_of(n), 256, 0, st>>>(blocks, flag, pos, n, cur_xyz, cur_old);
  LGF_HIP_CHECK(hipGetLastError());
  int64_t total = 0;
  for (int l = 0; m > 0; ++l) {
    if (total + m <= cap && out_blocks && out_levels) {
      copy_out_kernel<<<grid_of(m), 256, 0, st>>>(cur_xyz, m, l, out_blocks + 3 * total, out_levels + total);
      LGF_HIP_CHECK(hipGetLastError());
    }
    total += m;
    if (l + 1 >= kMaxLevels) break;
    int32_t *fl = nullptr, *rk = nullptr;
    LGF_HIP_CHECK(buf.get(&fl, m));
    LGF_HIP_CHECK(buf.get(&rk, m + 1));
    level_flags_kernel<<<grid_of(m), 256, 0, st>>>(cur_old, m, l, n_levels, omega, thr, fl);
    scan_kernel<<<1, 1024, 0, st>>>(fl, m, rk);
    LGF_HIP_CHECK(hipGetLastError());
    int32_t nf = 0;
    LGF_HIP_CHECK(hipMemcpyAsync(&nf, rk + m, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    LGF_HIP_CHECK(hipStreamSynchronize(st));
    const int64_t m2 = 8 * (int64_t)nf;
    if (m2 == 0) break;
    int32_t *nxt_xyz = nullptr, *nxt_old = nullptr;
    LGF_HIP_CHECK(buf.get(&nxt_xyz, 3 * m2));
    LGF_HIP_CHECK(buf.get(&nxt_old, m2));
    emit_children_kernel<<<grid_of(8 * m), 256, 0, st>>>(cur_xyz, fl, rk, m, l, keys, vals, tsize - 1, nxt_xyz,
                                                        nxt_old);
    LGF_HIP_CHECK(hipGetLastError());
    cur_xyz = nxt_xyz;
    cur_old = nxt_old;
    m = m2;
  }
  LGF_HIP_CHECK(hipStreamSynchronize(st));
  *n_out = total;
  return total <= cap ? hipSuccess : hipErrorOutOfMemory;
}

}  // namespace lgf
