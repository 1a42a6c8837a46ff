// Plan construction and step execution (host side).
//
// Per refinement level l (Sec. 3, Algorithm 2) the plan holds up to two FMM instances over the
// octree of that level's blocks (Sec. 2.1): channel T (all blocks are sources, all are targets:
// the total field of eq. amr_convs for leaf targets) and channel A (leaf blocks are sources,
// non-leaf blocks are targets: the leaf-only field passed to level l+1).  Both use the same tree,
// so A equals the paper's "FMM of all sources minus FMM of non-leaf sources".
//
// Tree: level k+1 holds floor(b/2) of level k; it stops at the first level whose nodes are all
// mutual neighbours (no influence list can be non-empty above it).  Lists: N(B) (Chebyshev
// distance <= 1, base level only) and I(B) (distance >= 2, parents neighbours), Fig. fmm_regions.
#include "plan.hpp"

#include <algorithm>
#include <limits>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <set>
#include <tuple>
#include <unordered_map>

namespace lgf {

namespace {

struct I3 {
  int x, y, z;
  bool operator==(const I3& o) const { return x == o.x && y == o.y && z == o.z; }
  bool operator<(const I3& o) const {
    if (z != o.z) return z < o.z;
    if (y != o.y) return y < o.y;
    return x < o.x;
  }
};
struct I3Hash {
  size_t operator()(const I3& a) const {
    uint64_t h = (uint64_t)(uint32_t)a.x * 0x9E3779B97F4A7C15ull;
    h ^= (uint64_t)(uint32_t)a.y * 0xC2B2AE3D27D4EB4Full + (h << 6) + (h >> 2);
    h ^= (uint64_t)(uint32_t)a.z * 0x165667B19E3779F9ull + (h << 6) + (h >> 2);
    return (size_t)h;
  }
};
using I3Map = std::unordered_map<I3, int, I3Hash>;

inline int floordiv2(int v) { return v >= 0 ? v / 2 : -((-v + 1) / 2); }
inline int floordiv(int v, int d) { return v >= 0 ? v / d : -((-v + d - 1) / d); }
inline I3 parent_of(I3 a) { return {floordiv2(a.x), floordiv2(a.y), floordiv2(a.z)}; }
inline int octant_of(I3 a) {
  const I3 p = parent_of(a);
  return (a.x - 2 * p.x) + 2 * (a.y - 2 * p.y) + 4 * (a.z - 2 * p.z);
}
inline int cheb(I3 a, I3 b) {
  return std::max(std::abs(a.x - b.x), std::max(std::abs(a.y - b.y), std::abs(a.z - b.z)));
}

// ----------------------------------------------------------------------------- 1-D weights
// Lagrange stencil for coordinate x (parent node units): n_i nodes, even counts around the
// bracketing pair, odd counts centred on the nearest node, shifted inside [0, nb-1].
void lagrange_row(double x, int n_i, int nb, int* lo_out, double* w) {
  int lo = (n_i % 2 == 0) ? (int)std::floor(x) - n_i / 2 + 1 : (int)std::floor(x + 0.5) - (n_i - 1) / 2;
  lo = std::min(std::max(lo, 0), nb - n_i);
  for (int j = 0; j < n_i; ++j) {
    double v = 1.0;
    for (int m = 0; m < n_i; ++m)
      if (m != j) v *= (x - double(lo + m)) / double(j - m);
    w[j] = v;
  }
  *lo_out = lo;
}

std::vector<double> lagrange_matrix(int nb, int n_i) {
  std::vector<double> W((size_t)2 * nb * nb, 0.0);
  std::vector<double> w(n_i);
  for (int j = 0; j < 2 * nb; ++j) {
    int lo;
    lagrange_row(j / 2.0 - 0.25, n_i, nb, &lo, w.data());
    for (int m = 0; m < n_i; ++m) W[(size_t)j * nb + lo + m] = w[m];
  }
  return W;
}

std::vector<double> refine_table(int nb) {
  std::vector<double> t((size_t)(2 * nb + 2) * 4);
  double w[3];
  for (int j = -1; j <= 2 * nb; ++j) {
    int lo;
    lagrange_row(j / 2.0 - 0.25, 3, nb, &lo, w);
    double* r = &t[(size_t)(j + 1) * 4];
    r[0] = lo; r[1] = w[0]; r[2] = w[1]; r[3] = w[2];
  }
  return t;
}

// ----------------------------------------------------------------------------- FMM instance
struct OctLevel {
  std::vector<I3> nodes;
  I3Map index;
  std::vector<int> parent;             // index into the next level
  std::vector<char> is_src, is_tgt, has_ifft, has_val, referenced, need_src;
  std::vector<int> src_slot, tgt_slot;
};

struct TileDesc {
  int k;
  int W;                               // targets per row: 8 or 4
  I3 key;                              // (x window, y pair, z pair)
  int tgt_node[4][kMacL];
  int src_node[36][kMacSlots];
  uint64_t mask;
};

struct Fmm {
  std::vector<OctLevel> lv;
  std::vector<TileDesc> rows;
  int64_t interactions = 0;
  std::vector<int64_t> level_interactions;
};

// valid offset d = t - src for target parity c (per dimension): c-3 <= d <= c+2
inline bool parity_ok(int d, int c) { return d >= c - 3 && d <= c + 2; }

void fmm_build(const std::vector<I3>& base, const std::vector<char>& src, const std::vector<char>& tgt,
               Fmm& F) {
  F.lv.clear();
  F.lv.emplace_back();
  {
    OctLevel& L0 = F.lv[0];
    L0.nodes = base;
    for (size_t i = 0; i < base.size(); ++i) L0.index[base[i]] = (int)i;
    L0.is_src = src;
    L0.is_tgt = tgt;
  }
  auto extent = [](const std::vector<I3>& v) {
    I3 lo = v[0], hi = v[0];
    for (const I3& a : v) {
      lo = {std::min(lo.x, a.x), std::min(lo.y, a.y), std::min(lo.z, a.z)};
      hi = {std::max(hi.x, a.x), std::max(hi.y, a.y), std::max(hi.z, a.z)};
    }
    return std::max(hi.x - lo.x, std::max(hi.y - lo.y, hi.z - lo.z));
  };
  while (extent(F.lv.back().nodes) > 1) {
    OctLevel& cur = F.lv.back();
    std::vector<I3> par;
    par.reserve(cur.nodes.size());
    for (const I3& a : cur.nodes) par.push_back(parent_of(a));
    std::sort(par.begin(), par.end());
    par.erase(std::unique(par.begin(), par.end()), par.end());
    OctLevel nxt;
    nxt.nodes = par;
    for (size_t i = 0; i < par.size(); ++i) nxt.index[par[i]] = (int)i;
    nxt.is_src.assign(par.size(), 0);
    nxt.is_tgt.assign(par.size(), 0);
    cur.parent.resize(cur.nodes.size());
    for (size_t i = 0; i < cur.nodes.size(); ++i) {
      const int pi = nxt.index.at(parent_of(cur.nodes[i]));
      cur.parent[i] = pi;
      if (cur.is_src[i]) nxt.is_src[pi] = 1;
      if (cur.is_tgt[i]) nxt.is_tgt[pi] = 1;
    }
    F.lv.push_back(std::move(nxt));
  }
  const int K = (int)F.lv.size();
  F.level_interactions.assign(K, 0);
  // rows, interactions, referenced sources
  for (int k = 0; k < K; ++k) {
    OctLevel& L = F.lv[k];
    const size_t n = L.nodes.size();
    L.has_ifft.assign(n, 0);
    L.referenced.assign(n, 0);
    const bool base_level = (k == 0);
    std::map<I3, TileDesc> rows8, rows4;
    for (size_t t = 0; t < n; ++t) {
      if (!L.is_tgt[t]) continue;
      const I3 a = L.nodes[t];
      const int cx = a.x & 1, cy = a.y & 1, cz = a.z & 1;
      int64_t cnt = 0;
      for (int dz = cz - 3; dz <= cz + 2; ++dz)
        for (int dy = cy - 3; dy <= cy + 2; ++dy)
          for (int dx = cx - 3; dx <= cx + 2; ++dx) {
            const bool near = std::abs(dx) <= 1 && std::abs(dy) <= 1 && std::abs(dz) <= 1;
            if (near && !base_level) continue;
            auto it = L.index.find({a.x - dx, a.y - dy, a.z - dz});
            if (it == L.index.end() || !L.is_src[it->second]) continue;
            L.referenced[it->second] = 1;
            ++cnt;
          }
      if (cnt == 0) continue;
      L.has_ifft[t] = 1;
      F.interactions += cnt;
      F.level_interactions[k] += cnt;
      // tiles of rows of 8 and of 4 targets (the planner picks one width per level)
      for (int wi = 0; wi < 2; ++wi) {
        const int W = wi == 0 ? kMacL : kMacL / 2;
        const int wx = floordiv(a.x, W), py = floordiv2(a.y), pz = floordiv2(a.z);
        const I3 key{wx, py, pz};
        auto& rows = wi == 0 ? rows8 : rows4;
        auto rit = rows.find(key);
        if (rit == rows.end()) {
          TileDesc r;
          r.k = k;
          r.W = W;
          r.key = key;
          for (int q = 0; q < 4; ++q)
            for (int i = 0; i < kMacL; ++i) r.tgt_node[q][i] = -1;
          r.mask = 0;
          for (int jz = 0; jz < 6; ++jz)
            for (int jy = 0; jy < 6; ++jy)
              for (int q = 0; q < kMacSlots; ++q) {
                auto it = q < W + 6 ? L.index.find({wx * W - 3 + q, 2 * py - 2 + jy, 2 * pz - 2 + jz})
                                    : L.index.end();
                const int id = (it != L.index.end() && L.is_src[it->second]) ? it->second : -1;
                r.src_node[jz * 6 + jy][q] = id;
                if (id >= 0) r.mask |= 1ull << (jz * 6 + jy);
              }
          rit = rows.emplace(key, r).first;
        }
        rit->second.tgt_node[(a.y - 2 * py) + 2 * (a.z - 2 * pz)][a.x - wx * W] = (int)t;
      }
    }
    for (auto& kv : rows8) F.rows.push_back(kv.second);
    for (auto& kv : rows4) F.rows.push_back(kv.second);
  }
  // values: top-down; source needs: top-down from referenced
  for (int k = K - 1; k >= 0; --k) {
    OctLevel& L = F.lv[k];
    const size_t n = L.nodes.size();
    L.has_val.assign(n, 0);
    L.need_src.assign(n, 0);
    for (size_t i = 0; i < n; ++i) {
      const bool pv = (k + 1 < K) && F.lv[k + 1].has_val[L.parent[i]];
      const bool pn = (k + 1 < K) && F.lv[k + 1].need_src[L.parent[i]];
      L.has_val[i] = L.is_tgt[i] && (L.has_ifft[i] || pv);
      L.need_src[i] = L.is_src[i] && (L.referenced[i] || pn);
    }
    L.src_slot.assign(n, -1);
    L.tgt_slot.assign(n, -1);
  }
}

// ----------------------------------------------------------------------------- device memory
void* fake_alloc(Plan* p, size_t bytes) {
  if (!p->next_fake) p->next_fake = (uintptr_t)1 << 44;
  void* q = (void*)p->next_fake;
  p->next_fake += (bytes + 2 * 4096 + 4095) / 4096 * 4096;     // guard gap between ranges
  p->ranges.push_back({(uintptr_t)q, bytes});
  return q;
}

// Constants of the plan (device memory it owns for its lifetime; fake ranges in a dry build).
struct Arena {
  Plan* p;
  uint64_t budget;
  hipError_t alloc(void** ptr, size_t bytes) {
    *ptr = nullptr;
    if (bytes == 0) return hipSuccess;
    if (budget && (uint64_t)(p->bytes + (int64_t)bytes) > budget) return hipErrorOutOfMemory;
    if (p->dry) {
      *ptr = fake_alloc(p, bytes);
    } else {
      hipError_t e = hipMalloc(ptr, bytes);
      if (e != hipSuccess) return e;
      p->allocs.push_back(*ptr);
      p->ranges.push_back({(uintptr_t)*ptr, bytes});
    }
    p->bytes += (int64_t)bytes;
    return hipSuccess;
  }
};

// The solve workspace: virtual addresses kVBase + offset, 256-byte aligned (see Binding).
struct VArena {
  Plan* p;
  hipError_t alloc(void** ptr, size_t bytes) {
    *ptr = nullptr;
    if (bytes == 0) return hipSuccess;
    const int64_t off = (p->vnext + 255) / 256 * 256;
    if (off + (int64_t)bytes >= ((int64_t)1 << kVTagShift)) return hipErrorOutOfMemory;
    *ptr = (void*)(uintptr_t)(kVBase + (uint64_t)off);
    p->ranges.push_back({(uintptr_t)*ptr, bytes});
    p->vnext = off + (int64_t)bytes;
    return hipSuccess;
  }
  // the range reads as zero in every solve (cleared when a binding takes the plan's items)
  void zero(const void* ptr, size_t bytes) {
    if (bytes) p->zero.push_back({(int64_t)((uint64_t)(uintptr_t)ptr - kVBase), (int64_t)bytes});
  }
};

// spectra count and size of a kernel set (s == 0: the 27 super-block neighbour spectra)
// s >= 1: block kernels at scale s; s <= -1: super-block kernels at scale -s
inline int spec_count(int s) { return s < 0 ? 27 : 343; }
inline int64_t spec_size(int nb, int s) {
  const int64_t b = s < 0 ? 2 * nb : nb;
  return (2 * b) * (2 * b) * (b + 1);
}

// kernel spectra of (nb, s) for a plan: the shared cache, or fake ranges in a dry build
hipError_t plan_spectra(Plan* p, int nb, int s, const SpecSet** out) {
  const int cnt = spec_count(s);
  const size_t S = (size_t)spec_size(nb, s);
  if (!p->dry) {
    LGF_HIP_CHECK(spectra_for(p->ctx, nb, s, out));
    p->ranges.push_back({(uintptr_t)(*out)->d64, cnt * S * sizeof(c64)});
    p->ranges.push_back({(uintptr_t)(*out)->d32, cnt * S * sizeof(c32)});
    p->ranges.push_back({(uintptr_t)(*out)->kp64, cnt * sizeof(void*)});
    p->ranges.push_back({(uintptr_t)(*out)->kp32, cnt * sizeof(void*)});
    if (s < 0) {
      p->ranges.push_back({(uintptr_t)(*out)->col64, 14 * S * sizeof(c64)});
      p->ranges.push_back({(uintptr_t)(*out)->col32, 14 * S * sizeof(c32)});
    }
    return hipSuccess;
  }
  auto key = std::make_pair(nb, s);
  auto it = p->dry_spectra.find(key);
  if (it == p->dry_spectra.end()) {
    SpecSet ss;
    ss.nb = nb;
    ss.s = s;
    ss.count = cnt;
    ss.spec = (int64_t)S;
    ss.d64 = (c64*)fake_alloc(p, cnt * S * sizeof(c64));
    ss.d32 = (c32*)fake_alloc(p, cnt * S * sizeof(c32));
    ss.kp64 = (const c64**)fake_alloc(p, cnt * sizeof(void*));
    ss.kp32 = (const c32**)fake_alloc(p, cnt * sizeof(void*));
    if (s < 0) {
      ss.col64 = (c64*)fake_alloc(p, 14 * S * sizeof(c64));
      ss.col32 = (c32*)fake_alloc(p, 14 * S * sizeof(c32));
    }
    it = p->dry_spectra.emplace(key, ss).first;
  }
  *out = &it->second;
  return hipSuccess;
}

}  // namespace

// ----------------------------------------------------------------------------- device context
namespace {
std::mutex g_ctx_mu;
std::map<int, DeviceCtx*> g_ctx;
}  // namespace

hipError_t device_ctx(DeviceCtx** out) {
  int dev = 0;
  LGF_HIP_CHECK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_ctx_mu);
  auto it = g_ctx.find(dev);
  if (it != g_ctx.end()) {
    *out = it->second;
    return hipSuccess;
  }
  DeviceCtx* c = new DeviceCtx();
  c->device = dev;
  LGF_HIP_CHECK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
  const size_t cube_n = (size_t)(kTableKmax + 1) * (kTableKmax + 1) * (kTableKmax + 1);
  LGF_HIP_CHECK(hipMalloc(&c->cube, cube_n * sizeof(double)));
  LGF_HIP_CHECK(hipMemsetAsync(c->cube, 0, cube_n * sizeof(double), c->stream));
  std::vector<int16_t> tri;
  for (int a = 0; a <= kTableKmax; ++a)
    for (int b = 0; b <= a; ++b)
      for (int cc = 0; cc <= b; ++cc)
        if (a * a + b * b + cc * cc <= 10000) {
          tri.push_back((int16_t)a);
          tri.push_back((int16_t)b);
          tri.push_back((int16_t)cc);
        }
  const int ntri = (int)(tri.size() / 3);
  double *nodes = nullptr, *wts = nullptr;
  int16_t* d_tri = nullptr;
  const int nq = quad_nodes();
  LGF_HIP_CHECK(hipMalloc(&nodes, (size_t)nq * (kTableKmax + 1) * sizeof(double)));
  LGF_HIP_CHECK(hipMalloc(&wts, (size_t)nq * sizeof(double)));
  LGF_HIP_CHECK(hipMalloc(&d_tri, tri.size() * sizeof(int16_t)));
  LGF_HIP_CHECK(hipMemcpyAsync(d_tri, tri.data(), tri.size() * sizeof(int16_t), hipMemcpyHostToDevice,
                               c->stream));
  LGF_HIP_CHECK(launch_green_table(c->cube, nodes, wts, d_tri, ntri, c->stream));
  LGF_HIP_CHECK(hipStreamSynchronize(c->stream));
  (void)hipFree(nodes);
  (void)hipFree(wts);
  (void)hipFree(d_tri);
  c->bytes = (int64_t)(cube_n * sizeof(double));
  g_ctx[dev] = c;
  *out = c;
  return hipSuccess;
}

hipError_t spectra_for(DeviceCtx* ctx, int nb, int s, const SpecSet** out) {
  std::lock_guard<std::mutex> lk(ctx->mu);
  auto key = std::make_pair(nb, s);
  auto it = ctx->spectra.find(key);
  if (it != ctx->spectra.end()) {
    *out = &it->second;
    return hipSuccess;
  }
  // s <= -1: kernels between neighbouring super-blocks of 2 nb cells at scale -s
  const int cnt = spec_count(s), R = s < 0 ? 1 : 3;
  const int bf = s < 0 ? 2 * nb : nb, sf = s < 0 ? -s : s;
  const int P = 2 * bf, H = bf + 1;
  const size_t S = (size_t)P * P * H, P3 = (size_t)P * P * P;
  std::vector<int32_t> sd;
  for (int dz = -R; dz <= R; ++dz)
    for (int dy = -R; dy <= R; ++dy)
      for (int dx = -R; dx <= R; ++dx) {
        sd.push_back(sf); sd.push_back(dx); sd.push_back(dy); sd.push_back(dz);
      }
  SpecSet ss;
  ss.nb = nb;
  ss.s = s;
  ss.count = cnt;
  ss.spec = (int64_t)S;
  int32_t* d_sd = nullptr;
  double* d_real = nullptr;
  c64* d_tmp = nullptr;
  LGF_HIP_CHECK(hipMalloc(&d_sd, sd.size() * sizeof(int32_t)));
  LGF_HIP_CHECK(hipMalloc(&d_real, cnt * P3 * sizeof(double)));
  LGF_HIP_CHECK(hipMalloc(&d_tmp, cnt * S * sizeof(c64)));
  LGF_HIP_CHECK(hipMalloc(&ss.d64, cnt * S * sizeof(c64)));
  LGF_HIP_CHECK(hipMalloc(&ss.d32, cnt * S * sizeof(c32)));
  LGF_HIP_CHECK(hipMalloc(&ss.kp64, cnt * sizeof(void*)));
  LGF_HIP_CHECK(hipMalloc(&ss.kp32, cnt * sizeof(void*)));
  LGF_HIP_CHECK(hipMemcpyAsync(d_sd, sd.data(), sd.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                               ctx->stream));
  LGF_HIP_CHECK(launch_kernel_spectra(bf, cnt, d_sd, ctx->cube, d_real, d_tmp, ss.d64, ss.d32, ctx->stream));
  std::vector<const void*> p64(cnt), p32(cnt);
  for (int i = 0; i < cnt; ++i) {
    p64[i] = ss.d64 + i * S;
    p32[i] = ss.d32 + i * S;
  }
  LGF_HIP_CHECK(hipMemcpyAsync((void*)ss.kp64, p64.data(), cnt * sizeof(void*), hipMemcpyHostToDevice, ctx->stream));
  LGF_HIP_CHECK(hipMemcpyAsync((void*)ss.kp32, p32.data(), cnt * sizeof(void*), hipMemcpyHostToDevice, ctx->stream));
  if (s < 0) {
    // kernel columns of the fused near step: the 14 kernels h <= 13, [h][line][kz]
    LGF_HIP_CHECK(hipMalloc(&ss.col64, 14 * S * sizeof(c64)));
    LGF_HIP_CHECK(hipMalloc(&ss.col32, 14 * S * sizeof(c32)));
    LGF_HIP_CHECK(launch_kernel_columns<double>(nb, ss.d64, ss.col64, ctx->stream));
    LGF_HIP_CHECK(launch_kernel_columns<float>(nb, ss.d32, ss.col32, ctx->stream));
    ctx->bytes += (int64_t)(14 * S * (sizeof(c64) + sizeof(c32)));
  }
  LGF_HIP_CHECK(hipStreamSynchronize(ctx->stream));
  (void)hipFree(d_sd);
  (void)hipFree(d_real);
  (void)hipFree(d_tmp);
  ctx->bytes += (int64_t)(cnt * S * (sizeof(c64) + sizeof(c32)));
  auto res = ctx->spectra.emplace(key, ss);
  *out = &res.first->second;
  return hipSuccess;
}

// ----------------------------------------------------------------------------- plan build
namespace {

struct HostItems {
  std::vector<uint8_t> buf;
  template <typename X> size_t add(const std::vector<X>& v) {
    size_t off = (buf.size() + 255) / 256 * 256;
    buf.resize(off + v.size() * sizeof(X));
    if (!v.empty()) std::memcpy(buf.data() + off, v.data(), v.size() * sizeof(X));
    return off;
  }
};

struct PendingStep {
  int l, phase, sub, kind, ty;
  size_t off;
  int32_t count;
  const double* w;
  int64_t work;
  int mode;
  int chain;
  bool lds = false;
};

// ----------------------------------------------------------------------------- item validation
bool in_ranges(const Plan* p, const void* ptr, size_t len) {
  const uintptr_t a = (uintptr_t)ptr;
  for (const auto& r : p->ranges)
    if (a >= r.first && a + len <= r.first + r.second) return true;
  return false;
}

struct SlotCounts {
  int64_t nsrc[2], ntgt[2];            // block spectra slots per element type (source: + zero slot)
  int64_t nsup_src[2], nsup_tgt[2];    // super-block spectra slots
};

// Checks every item of a step (slots in range, pointers inside the plan's ranges) and records, in
// *rel, the 8-byte words of the item image (starting at image) that hold a workspace address.
bool validate_step(const Plan* p, int kind, int ty, int mode, const uint8_t* items, int count, int64_t n,
                   const SlotCounts& sc, std::string* err, const uint8_t* image, std::set<uint32_t>* rel) {
  const int nb = p->nb;
  const size_t N3 = (size_t)nb * nb * nb;
  const size_t S = (size_t)(2 * nb) * (2 * nb) * (nb + 1);
  const size_t S2 = (size_t)spec_size(nb, -1);
  const size_t TMP2 = (size_t)(2 * nb) * (4 * nb) * (2 * nb + 1);    // intermediate z-plane stack
  const int64_t* nsrc = sc.nsrc;
  const int64_t* ntgt = sc.ntgt;
  const size_t es = ty == 0 ? 4 : 8, esc = ty == 1 ? 8 : 4, esp = ty == 0 ? 4 : 8;  // MIX: child 4, parent 8
  const bool child_in_ok = ty == 1;                    // FP64 children may come from the input
  const int64_t nmax = n * (int64_t)N3;
  auto bad = [&](const char* what, int i) {
    if (err) *err = std::string("internal plan check failed: ") + what + " (kind " + std::to_string(kind) +
                    ", item " + std::to_string(i) + ")";
    return false;
  };
  auto off_ok = [&](int64_t o) { return o >= 0 && o % (int64_t)N3 == 0 && o + (int64_t)N3 <= nmax; };
  // a pointer field: inside the plan's ranges; a workspace address is recorded for relocation
  auto rg = [&](const auto& field, size_t len) {
    const uint64_t v = (uint64_t)(uintptr_t)field;
    if ((v >> kVTagShift) == (kVBase >> kVTagShift))
      rel->insert((uint32_t)(((const uint8_t*)&field - image) / 8));
    return in_ranges(p, (const void*)field, len);
  };
  for (int i = 0; i < count; ++i) {
    switch (kind) {
      case K_FWD: {
        const auto& it = ((const FftFwdItem<double>*)items)[i];
        if (!rg(it.src, N3 * es) || !rg(it.dst, 2 * S * es)) return bad("fft_fwd", i);
        break;
      }
      case K_INV: {
        const auto& it = ((const FftInvItem<double>*)items)[i];
        if (!rg(it.src, 2 * S * es) || !rg(it.dst, N3 * es)) return bad("fft_inv", i);
        break;
      }
      case K_MAC: {
        const auto& it = ((const MacTile<double>*)items)[i];
        const int t = ty == 0 ? 0 : 1;
        for (int j = 0; j < 36; ++j)
          for (int q = 0; q < kMacSlots; ++q)
            if (it.src[j][q] < 0 || it.src[j][q] > nsrc[t]) return bad("mac source slot", i);
        const int w = (mode & kMacHalfRows) ? kMacL / 2 : kMacL;
        for (int r = 0; r < 4; ++r)
          for (int q = 0; q < kMacL; ++q)
            if (it.tgt[r][q] < -1 || it.tgt[r][q] >= ntgt[t] || (q >= w && it.tgt[r][q] != -1))
              return bad("mac target slot", i);
        if (!rg(it.fhat, (nsrc[t] + 1) * 2 * S * es)) return bad("mac source arena", i);
        if (ntgt[t] && !rg(it.uhat, ntgt[t] * 2 * S * es)) return bad("mac target arena", i);
        if (!rg(it.kptr, 343 * sizeof(void*))) return bad("mac kernel table", i);
        if ((mode & (kMacHalfRows - 1)) == kMacLds) {      // LDS form: rows of 4, compact slots
          if (!(mode & kMacHalfRows) || it.src_n < 1 || it.src_n > kMacLdsSrc || it.src_lo < 0 ||
              it.src_lo + it.src_n > nsrc[t])
            return bad("mac lds source range", i);
          for (int j = 0; j < 36; ++j)
            for (int q = 0; q < kMacSlots; ++q)
              if (it.src[j][q] != nsrc[t] && (it.src[j][q] < it.src_lo || it.src[j][q] >= it.src_lo + it.src_n))
                return bad("mac lds source slot", i);
        }
        break;
      }
      case K_ANTERP: {
        const auto& it = ((const AnterpItem<double, double>*)items)[i];
        if (!rg(it.dst, N3 * esp)) return bad("anterp parent", i);
        for (int c = 0; c < 8; ++c) {
          if (it.child[c] && !rg(it.child[c], N3 * esc)) return bad("anterp child", i);
          if (it.child_in[c] != -1 && (it.child[c] || !child_in_ok || !off_ok(it.child_in[c])))
            return bad("anterp child offset", i);
        }
        break;
      }
      case K_INTERP: {
        const auto& it = ((const InterpItem<double, double>*)items)[i];
        if (!rg(it.child, N3 * esc) || !rg(it.parent, N3 * esp)) return bad("interp", i);
        if (it.octant < 0 || it.octant > 7) return bad("interp octant", i);
        break;
      }
      case K_COMBINE: {
        const auto& it = ((const CombineItem<double>*)items)[i];
        if (it.dst_d ? !rg(it.dst_d, N3 * 8) : !off_ok(it.dst_out)) return bad("combine dst", i);
        if (it.v && !rg(it.v, N3 * es)) return bad("combine v", i);
        if (it.far && !rg(it.far, N3 * es)) return bad("combine far", i);
        if (it.base && !rg(it.base, N3 * 8)) return bad("combine base", i);
        break;
      }
      case K_CONVERT: {
        const auto& it = ((const ConvertItem<double>*)items)[i];
        if (!rg(it.dst, N3 * es)) return bad("convert dst", i);
        if (it.src ? !rg(it.src, N3 * 8) : !off_ok(it.src_in)) return bad("convert src", i);
        break;
      }
      case K_COARSEN: {
        const auto& it = ((const CoarsenItem*)items)[i];
        if (!rg(it.dst, N3 * 8)) return bad("coarsen dst", i);
        for (int c = 0; c < 8; ++c)
          if (it.child[c] ? !rg(it.child[c], N3 * 8) : !off_ok(it.child_in[c])) return bad("coarsen child", i);
        break;
      }
      case K_REFINE: {
        const auto& it = ((const RefineItem*)items)[i];
        if (!rg(it.jw, N3 * 8) || !rg(it.parent_w, N3 * 8)) return bad("refine", i);
        break;
      }
      case K_CORRECT: {
        const auto& it = ((const CorrectItem<double>*)items)[i];
        if (!rg(it.g, N3 * es) || !rg(it.jw, N3 * 8) || !rg(it.parent_w, N3 * 8))
          return bad("correct", i);
        if (it.f ? !rg(it.f, N3 * 8) : !off_ok(it.f_in)) return bad("correct f", i);
        for (int f = 0; f < 6; ++f)
          if (it.nbr[f] && !rg(it.nbr[f], N3 * 8)) return bad("correct neighbour", i);
        break;
      }
      case K_RESIDUAL: {
        const auto& it = ((const ResidualItem*)items)[i];
        if ((it.r && !rg(it.r, N3 * 8)) || (it.conv && !rg(it.conv, N3 * 4)) || !off_ok(it.off))
          return bad("residual", i);
        for (int f = 0; f < 6; ++f)
          if (it.nbr_off[f] != -1 && !off_ok(it.nbr_off[f])) return bad("residual neighbour", i);
        break;
      }
      case K_SUP_FWD: {
        const auto& it = ((const SuperFwdItem<double>*)items)[i];
        if (!rg(it.dst, 2 * S2 * es) || !rg(it.tmp, 2 * TMP2 * es)) return bad("super fwd", i);
        for (int c = 0; c < 8; ++c) {
          if (it.child[c] && !rg(it.child[c], N3 * esc)) return bad("super fwd child", i);
          if (it.child_in[c] != -1 && (it.child[c] || !child_in_ok || !off_ok(it.child_in[c])))
            return bad("super fwd child offset", i);
        }
        break;
      }
      case K_SUP_INV: {
        const auto& it = ((const SuperInvItem<double>*)items)[i];
        if (!rg(it.src, 2 * S2 * es) || !rg(it.tmp, 2 * TMP2 * es)) return bad("super inv", i);
        for (int c = 0; c < 8; ++c)
          if (it.child[c] && !rg(it.child[c], N3 * esc)) return bad("super inv child", i);
        break;
      }
      case K_NEAR_MAC: {
        const int t = ty == 0 ? 0 : 1;
        if (near_compact(mode)) {
          const auto& it = ((const NearCTile<double>*)items)[i];
          if (near_fused(mode) && !rg(it.ktr, 14 * S2 * es)) return bad("near fused kernel columns", i);
          const int rz = near_ctile_rz(mode), cap = near_ctile_cap(mode);
          if (it.rz != rz) return bad("near pipelined tile shape", i);
          if (it.nreal < 0 || it.nreal > cap || it.zero != sc.nsup_src[t]) return bad("near pipelined tile entries", i);
          for (int j = 0; j < 4 * (rz + 2) * (kTileW + 2); ++j) {
            const int x = j % (kTileW + 2);
            if (!it.edges && (x == 0 || x == kTileW + 1) && it.loff[j] != (uint32_t)(cap * 64))
              return bad("near pipelined tile edges", i);
          }
          for (int e = 0; e < kCTileCapMax; ++e)
            if (it.src[e] < 0 || it.src[e] > sc.nsup_src[t] || (e < it.nreal && it.src[e] == it.zero))
              return bad("near pipelined tile source slot", i);
          for (int j = 0; j < kTileSrcRowsMax * (kTileW + 2); ++j) {
            const uint32_t o = it.loff[j];
            if (o % 64 || (o / 64 >= (uint32_t)it.nreal && o / 64 != (uint32_t)cap)) return bad("near pipelined tile offset", i);
          }
          for (int r = 0; r < kTileRowsMax; ++r)
            for (int q = 0; q < kMacL; ++q)
              if (it.tgt[r][q] < -1 || it.tgt[r][q] >= sc.nsup_tgt[t]) return bad("near tile target slot", i);
          // 16-byte copies straight into LDS: the arena must be 16-byte aligned
          if ((uintptr_t)it.fhat % 16) return bad("near pipelined tile alignment", i);
          if (!rg(it.fhat, (sc.nsup_src[t] + 1) * 2 * S2 * es)) return bad("near source arena", i);
          if (sc.nsup_tgt[t] && !rg(it.uhat, sc.nsup_tgt[t] * 2 * S2 * es)) return bad("near target arena", i);
          if (!rg(it.kptr, 27 * sizeof(void*))) return bad("near kernel table", i);
          break;
        }
        if (mode > kNearTiled) {
          const auto& it = ((const NearTile<double>*)items)[i];
          if (!(mode == kNearTiled + 4 && it.rz == 2) && !(mode == kNearTiled + 6 && it.rz == 4))
            return bad("near tile shape", i);
          for (int j = 0; j < 4 * (it.rz + 2) * (kTileW + 2); ++j)
            if (it.src[j] < 0 || it.src[j] > sc.nsup_src[t]) return bad("near tile source slot", i);
          for (int r = 0; r < kTileRowsMax; ++r)
            for (int q = 0; q < kMacL; ++q)
              if (it.tgt[r][q] < -1 || it.tgt[r][q] >= sc.nsup_tgt[t]) return bad("near tile target slot", i);
          if (!rg(it.fhat, (sc.nsup_src[t] + 1) * 2 * S2 * es)) return bad("near source arena", i);
          if (sc.nsup_tgt[t] && !rg(it.uhat, sc.nsup_tgt[t] * 2 * S2 * es)) return bad("near target arena", i);
          if (!rg(it.kptr, 27 * sizeof(void*))) return bad("near kernel table", i);
          break;
        }
        if (mode != 2 && mode != 4 && mode != 8) return bad("near row width", i);
        const auto& it = ((const NearRow<double>*)items)[i];
        if (it.ngroups < 0 || it.ngroups > 3) return bad("near row groups", i);
        for (int j = 0; j < 9; ++j) {
          if (((it.pj_code >> (4 * j)) & 15u) > 8) return bad("near source row index", i);
          for (int q = 0; q < kNearSlots; ++q)
            if (it.src[j][q] < 0 || it.src[j][q] > sc.nsup_src[t]) return bad("near source slot", i);
        }
        for (int q = 0; q < kMacL; ++q)
          if (it.tgt[q] < -1 || it.tgt[q] >= sc.nsup_tgt[t]) return bad("near target slot", i);
        if (!rg(it.fhat, (sc.nsup_src[t] + 1) * 2 * S2 * es)) return bad("near source arena", i);
        if (sc.nsup_tgt[t] && !rg(it.uhat, sc.nsup_tgt[t] * 2 * S2 * es)) return bad("near target arena", i);
        if (!rg(it.kptr, 27 * sizeof(void*))) return bad("near kernel table", i);
        break;
      }
      default:
        return bad("unknown kind", i);
    }
  }
  return true;
}

// Element type of octree level k: the FP32 mode runs the base level of every refinement level
// in FP32 and the coarse (far-field) levels in FP64; the FP64 mode runs everything in FP64.
// Items are built with the <double> layouts, which are identical to the <float> ones (only
// pointers change type); each step records the element type its kernel is instantiated for.
enum : int { TY_F32 = 0, TY_F64 = 1, TY_MIX = 2 };   // TY_MIX: FP32 child level, FP64 parent level

}  // namespace
void sync_super_modes(Plan* p);
namespace {

hipError_t build_plan(Plan* p, const std::vector<I3>& coords, const std::vector<int>& lev,
                      uint64_t budget, std::string* err) {
  const int nb = p->nb;
  const int64_t N3 = (int64_t)nb * nb * nb;
  const int P = 2 * nb;
  const int64_t S = (int64_t)P * P * (nb + 1);
  const int64_t n = p->nblocks;
  const int LR = p->LR;
  const int tyb = p->fp32 ? TY_F32 : TY_F64;
  // coarse octree levels run in FP64 except in a correction plan (all FP32)
  auto ty_of = [&](int k) { return (k == 0 || p->all_fp32) ? tyb : TY_F64; };
  auto es = [](int ty) { return ty == TY_F32 ? (int64_t)4 : (int64_t)8; };
  Arena ar{p, budget};                 // constants
  VArena va{p};                        // solve workspace (virtual addresses)

  std::vector<std::vector<int>> ids(LR);
  for (int64_t i = 0; i < n; ++i) ids[lev[i]].push_back((int)i);
  std::vector<I3Map> cmap(LR);
  for (int l = 0; l < LR; ++l)
    for (int i : ids[l]) cmap[l][coords[i]] = i;
  std::vector<char> leaf(n, 1);
  for (int l = 0; l + 1 < LR; ++l)
    for (int i : ids[l]) {
      const I3 c = coords[i];
      if (cmap[l + 1].count({2 * c.x, 2 * c.y, 2 * c.z})) leaf[i] = 0;
    }
  auto child_of = [&](int i, int oc) {
    const I3 c = coords[i];
    return cmap[lev[i] + 1].at({2 * c.x + (oc & 1), 2 * c.y + ((oc >> 1) & 1), 2 * c.z + ((oc >> 2) & 1)});
  };
  auto face_nbr = [&](int i, int face) {
    I3 c = coords[i];
    const int ax = face >> 1, sg = (face & 1) ? 1 : -1;
    if (ax == 0) c.x += sg; else if (ax == 1) c.y += sg; else c.z += sg;
    auto it = cmap[lev[i]].find(c);
    return it == cmap[lev[i]].end() ? -1 : it->second;
  };

  // FMM instances and slots (per element type)
  std::vector<Fmm> chT(LR), chA(LR);
  std::vector<char> hasA(LR, 0);
  int64_t nsrc[2] = {0, 0}, ntgt[2] = {0, 0};
  std::vector<int> base_src_slot(n, -1);
  for (int l = 0; l < LR; ++l) {
    std::vector<I3> bc;
    std::vector<char> all(ids[l].size(), 1), lf(ids[l].size()), nl(ids[l].size());
    for (size_t a = 0; a < ids[l].size(); ++a) {
      bc.push_back(coords[ids[l][a]]);
      lf[a] = leaf[ids[l][a]];
      nl[a] = !leaf[ids[l][a]];
      if (nl[a]) hasA[l] = 1;
    }
    fmm_build(bc, all, all, chT[l]);
    if (hasA[l]) fmm_build(bc, lf, nl, chA[l]);
    for (size_t a = 0; a < ids[l].size(); ++a) {
      chT[l].lv[0].src_slot[a] = (int)nsrc[tyb];
      base_src_slot[ids[l][a]] = (int)nsrc[tyb];
      ++nsrc[tyb];
    }
    for (int ch = 0; ch < 2; ++ch) {
      if (ch == 1 && !hasA[l]) continue;
      Fmm& F = ch == 0 ? chT[l] : chA[l];
      for (size_t k = 0; k < F.lv.size(); ++k) {
        OctLevel& L = F.lv[k];
        const int ty = ty_of((int)k);
        for (size_t i = 0; i < L.nodes.size(); ++i) {
          if (k == 0 && L.is_src[i]) L.src_slot[i] = chT[l].lv[0].src_slot[i];
          else if (k > 0 && L.need_src[i]) L.src_slot[i] = (int)nsrc[ty]++;
          if (L.has_val[i]) L.tgt_slot[i] = (int)ntgt[ty]++;
        }
      }
    }
    p->Kmax = std::max(p->Kmax, (int)chT[l].lv.size());
  }

  // Base level as parent super-blocks (Sec. 2.1: a block's near list N(B) and influence list
  // I(B) together are the children of the 27 neighbours of its parent): per (refinement level,
  // channel) the whole base-level interaction is one zero-padded convolution per parent
  // super-block against its 27 neighbours.  Target super-blocks are the parents of blocks with
  // base-level interactions, source super-blocks their neighbours holding source children.  A
  // source super-block spectrum is computed once per distinct set of source children (channels
  // T and A share it where they agree).  Spectra arenas: 0 = FP32, 1 = FP64.  (The coarse
  // octree levels keep the block-wise influence lists: there a super-block convolution would
  // cover N(B) as well, which would have to be subtracted, and at their sizes the extra
  // transforms cost more than the tile MAC they replace.)
  struct SupTgt { I3 c; int slot; int child[8]; };
  struct SupInst { int l, ch, k, a; std::vector<SupTgt> tg; I3Map sslot; int64_t pairs = 0; };
  struct SupSrc { int l, k; std::array<int, 8> children; };
  std::vector<SupInst> sup;
  std::map<std::pair<int, std::array<int, 8>>, int> sup_src_of;   // (arena, child slots) -> slot
  std::vector<SupSrc> sup_src[2];                                  // per arena, by slot
  int64_t nsup_src[2] = {0, 0}, nsup_tgt[2] = {0, 0};
  // Super-block spectra of the base level: the base level's type on single-level layouts; FP64
  // spectra of FP32 blocks (TY_MIX) where the layout has refinement.  Defect correction forms
  // its residual only where all six neighbours are stored, so it cannot remove FP32 spectral
  // error at refinement interfaces: a block-smooth error there stays, and the correction spreads
  // it (by 3-4x in L-inf on the torus layouts), while on a single level only the outer boundary
  // is excluded.
  // A defect-correction re-solve computes a correction of the size of the FP32 error, whose own
  // FP32 rounding is negligible: its plan keeps FP32 spectra everywhere.
  const int tys = p->all_fp32 ? TY_F32 : (p->fp32 && LR > 1) ? TY_MIX : tyb;
  auto arena_of = [&](int k) { return (k == 0 && tys == TY_F32) ? 0 : 1; };
  auto sup_ty = [&](int k) { return k == 0 ? tys : TY_F64; };
  if (p->super_base) {
    for (int l = 0; l < LR; ++l)
      for (int ch = 0; ch < 2; ++ch) {
        if (ch == 1 && !hasA[l]) continue;
        const Fmm& F = ch == 0 ? chT[l] : chA[l];
        for (int k = 0; k < 1; ++k) {
          const OctLevel& L = F.lv[k];
          const int a = arena_of(k);
          auto is_source = [&](size_t i) { return (bool)L.is_src[i]; };
          std::unordered_map<I3, std::array<int, 8>, I3Hash> smap, tmap;
          const std::array<int, 8> none{-1, -1, -1, -1, -1, -1, -1, -1};
          bool any_tgt = false;
          for (size_t i = 0; i < L.nodes.size(); ++i) {
            const I3 par = parent_of(L.nodes[i]);
            const int oc = octant_of(L.nodes[i]);
            if (is_source(i)) smap.emplace(par, none).first->second[oc] = L.src_slot[i];
            if (L.has_ifft[i]) {
              tmap.emplace(par, none).first->second[oc] = (int)i;
              any_tgt = true;
            }
          }
          if (!any_tgt) continue;
          std::vector<I3> keys;
          for (const auto& kv : tmap) keys.push_back(kv.first);
          std::sort(keys.begin(), keys.end());
          SupInst si;
          si.l = l;
          si.ch = ch;
          si.k = k;
          si.a = a;
          for (const I3& T : keys) {
            SupTgt t;
            t.c = T;
            t.slot = (int)nsup_tgt[a]++;
            const std::array<int, 8>& kids = tmap.at(T);
            for (int oc = 0; oc < 8; ++oc) t.child[oc] = kids[oc];
            for (int dz = -1; dz <= 1; ++dz)
              for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                  const I3 Sx{T.x - dx, T.y - dy, T.z - dz};
                  auto it = smap.find(Sx);
                  if (it == smap.end()) continue;
                  ++si.pairs;
                  if (si.sslot.count(Sx)) continue;
                  const auto key = std::make_pair(a, it->second);
                  auto q = sup_src_of.find(key);
                  if (q == sup_src_of.end()) {
                    q = sup_src_of.emplace(key, (int)nsup_src[a]++).first;
                    sup_src[a].push_back({l, k, it->second});
                  }
                  si.sslot[Sx] = q->second;
                }
            si.tg.push_back(t);
          }
          sup.push_back(std::move(si));
        }
      }
  }

  // workspace arenas
  void* tmp = nullptr;
  if (LR > 1) {
    LGF_HIP_CHECK(va.alloc(&tmp, n * N3 * sizeof(double)));
    p->fe = (double*)tmp;
    LGF_HIP_CHECK(va.alloc(&p->jw, n * N3 * sizeof(double)));
    LGF_HIP_CHECK(va.alloc(&p->w, n * N3 * sizeof(double)));
  }
  uint8_t *srcA[2], *fhatA[2], *uhatA[2], *vA[2];
  for (int ty = 0; ty < 2; ++ty) {
    void *a = nullptr, *b = nullptr, *c = nullptr, *d = nullptr;
    LGF_HIP_CHECK(va.alloc(&a, nsrc[ty] * N3 * es(ty)));
    // one extra all-zero spectrum (slot nsrc[ty]) stands in for absent sources in MAC tiles;
    // the whole source-spectrum arena reads as zero before the pass writes it
    LGF_HIP_CHECK(va.alloc(&b, (nsrc[ty] + 1) * S * 2 * es(ty)));
    va.zero(b, (nsrc[ty] + 1) * S * 2 * es(ty));
    LGF_HIP_CHECK(va.alloc(&c, ntgt[ty] * S * 2 * es(ty)));
    LGF_HIP_CHECK(va.alloc(&d, ntgt[ty] * N3 * es(ty)));
    srcA[ty] = (uint8_t*)a; fhatA[ty] = (uint8_t*)b; uhatA[ty] = (uint8_t*)c; vA[ty] = (uint8_t*)d;
  }
  const int64_t S2 = spec_size(nb, -1);
  uint8_t* sfhA[2] = {nullptr, nullptr};
  uint8_t* suhA[2] = {nullptr, nullptr};
  for (int a = 0; a < 2; ++a) {
    if (!nsup_tgt[a]) continue;
    const int64_t ea = a == 0 ? 4 : 8;
    void *b = nullptr, *c = nullptr;
    LGF_HIP_CHECK(va.alloc(&b, (nsup_src[a] + 1) * S2 * 2 * ea));   // last slot: zero spectrum
    va.zero((uint8_t*)b + nsup_src[a] * S2 * 2 * ea, S2 * 2 * ea);
    LGF_HIP_CHECK(va.alloc(&c, nsup_tgt[a] * S2 * 2 * ea));
    sfhA[a] = (uint8_t*)b;
    suhA[a] = (uint8_t*)c;
  }
  p->sfhat = sfhA[arena_of(0)];
  p->suhat = suhA[arena_of(0)];
  p->src = srcA[tyb];
  p->fhat = fhatA[tyb];
  p->uhat = uhatA[tyb];
  p->v = vA[tyb];
  // With the super-block base level, the coarse field interpolated into a base block goes to an
  // array of its own (indexed like the block's level field) and the combine adds the two: the
  // interpolation then runs on the far-field chain, beside the super-block inverse transforms,
  // instead of after their join.
  uint8_t* farA = nullptr;
  if (p->super_base && ntgt[tyb]) {
    LGF_HIP_CHECK(va.alloc(&tmp, ntgt[tyb] * N3 * es(tyb)));
    farA = (uint8_t*)tmp;
  }
  std::vector<char> far_used(ntgt[tyb], 0);
  if (p->fp32 && p->dc_iters > 0 && LR > 1) {      // r of the finer levels' blocks (FP64)
    LGF_HIP_CHECK(va.alloc(&tmp, n * N3 * sizeof(double)));
    p->r = (double*)tmp;
  }
  p->ws_bytes = p->vnext;
  {
    const std::vector<double> W = lagrange_matrix(nb, p->n_i), W3 = refine_table(nb);
    // the refinement kernel stages nb/2 + 2 parent cells per axis from the stencil start of
    // the octant's first child cell
    for (int c = 0; c < 2; ++c)
      for (int j = 0; j < nb; ++j) {
        const int lo = (int)W3[4 * (c * nb + j + 1)], base = (int)W3[4 * (c * nb + 1)];
        if (lo < base || lo - base + 3 > nb / 2 + 2) {
          if (err) *err = "internal: refinement stencil outside the staged parent region";
          return hipErrorInvalidValue;
        }
      }
    LGF_HIP_CHECK(ar.alloc(&tmp, W.size() * sizeof(double)));
    p->d_w = (double*)tmp;
    if (!p->dry) LGF_HIP_CHECK(hipMemcpy(p->d_w, W.data(), W.size() * sizeof(double), hipMemcpyHostToDevice));
    LGF_HIP_CHECK(ar.alloc(&tmp, W3.size() * sizeof(double)));
    p->d_w3 = (double*)tmp;
    if (!p->dry) LGF_HIP_CHECK(hipMemcpy(p->d_w3, W3.data(), W3.size() * sizeof(double), hipMemcpyHostToDevice));
  }
  using D = double;
  auto SRC = [&](int ty, int64_t slot) { return (D*)(srcA[ty] + slot * N3 * es(ty)); };
  auto FH = [&](int ty, int64_t slot) { return (cpx<D>*)(fhatA[ty] + slot * S * 2 * es(ty)); };
  auto UH = [&](int ty, int64_t slot) { return (cpx<D>*)(uhatA[ty] + slot * S * 2 * es(ty)); };
  auto V = [&](int ty, int64_t slot) { return (D*)(vA[ty] + slot * N3 * es(ty)); };
  auto FAR = [&](int64_t slot) { return (D*)(farA + slot * N3 * es(tyb)); };
  auto SFH = [&](int a, int64_t slot) { return (cpx<D>*)(sfhA[a] + slot * S2 * 2 * (a == 0 ? 4 : 8)); };
  auto SUH = [&](int a, int64_t slot) { return (cpx<D>*)(suhA[a] + slot * S2 * 2 * (a == 0 ? 4 : 8)); };
  // Near rows: W targets along x at x0 = W wx, their 27 neighbours' spectra in groups of 3
  // non-empty source rows (zero slot where absent).  All rows of one call share fhat/uhat/kptr.
  auto make_rows = [&](const std::vector<std::pair<I3, int>>& tg, const I3Map& srcs, int zero, int W,
                       const cpx<D>* fhat, cpx<D>* uhat, const c64* const* kptr,
                       std::vector<NearRow<D>>& out) {
    std::map<I3, size_t> row_of;
    for (const auto& t : tg) {
      const int wx = floordiv(t.first.x, W);
      const I3 key{wx, t.first.y, t.first.z};
      auto it = row_of.find(key);
      if (it == row_of.end()) {
        NearRow<D> r{};
        for (int i = 0; i < kMacL; ++i) r.tgt[i] = -1;
        int nl = 0;                      // listed (non-empty) source rows
        for (int pj = 0; pj < 9; ++pj) {
          const int dz = pj / 3 - 1, dy = pj % 3 - 1;
          int slots[kNearSlots];
          bool any = false;
          for (int q = 0; q < kNearSlots; ++q) {
            auto sit = q < W + 2 ? srcs.find({wx * W - 1 + q, t.first.y - dy, t.first.z - dz}) : srcs.end();
            slots[q] = sit != srcs.end() ? sit->second : zero;
            any |= sit != srcs.end();
          }
          if (!any) continue;
          for (int q = 0; q < kNearSlots; ++q) r.src[nl][q] = slots[q];
          r.pj_code |= (uint64_t)pj << (4 * nl++);
        }
        for (int q = nl; q < 9; ++q)     // padding rows read the zero spectrum
          for (int x = 0; x < kNearSlots; ++x) r.src[q][x] = zero;
        r.ngroups = (nl + 2) / 3;
        r.fhat = fhat;
        r.uhat = uhat;
        r.kptr = kptr;
        it = row_of.emplace(key, out.size()).first;
        out.push_back(r);
      }
      out[it->second].tgt[t.first.x - wx * W] = t.second;
    }
  };
  // Near tiles: 2 x RZ rows of kTileW targets sharing their 4 x (RZ + 2) source rows (staged in
  // LDS)
  auto make_tiles = [&](const std::vector<std::pair<I3, int>>& tg, const I3Map& srcs, int zero,
                        const cpx<D>* fhat, cpx<D>* uhat, const cpx<D>* const* kptr,
                        std::vector<NearTile<D>>& out, int RZ = 2) {
    std::map<I3, size_t> tile_of;
    for (const auto& t : tg) {
      const int wx = floordiv(t.first.x, kTileW), ty2 = floordiv(t.first.y, 2), tz2 = floordiv(t.first.z, RZ);
      const I3 key{wx, ty2, tz2};
      auto it = tile_of.find(key);
      if (it == tile_of.end()) {
        NearTile<D> q{};
        for (int r = 0; r < kTileRowsMax; ++r)
          for (int i = 0; i < kMacL; ++i) q.tgt[r][i] = -1;
        for (int j = 0; j < kTileSrcRowsMax * (kTileW + 2); ++j) q.src[j] = zero;
        for (int qz = 0; qz < RZ + 2; ++qz)
          for (int qy = 0; qy < 4; ++qy)
            for (int x = 0; x < kTileW + 2; ++x) {
              auto sit = srcs.find({wx * kTileW - 1 + x, 2 * ty2 - 1 + qy, RZ * tz2 - 1 + qz});
              q.src[(qy + 4 * qz) * (kTileW + 2) + x] = sit != srcs.end() ? sit->second : zero;
              if (sit != srcs.end()) q.src_mask |= 1u << (qy + 4 * qz);
            }
        q.zero = zero;
        q.rz = RZ;
        q.fhat = fhat;
        q.uhat = uhat;
        q.kptr = kptr;
        it = tile_of.emplace(key, out.size()).first;
        out.push_back(q);
      }
      const int r = (t.first.y - 2 * ty2) + 2 * (t.first.z - RZ * tz2);
      out[it->second].tgt[r][t.first.x - wx * kTileW] = t.second;
      out[it->second].row_mask |= 1u << r;
    }
  };
  // compact tiles for the pipelined form: the same tiles staging only the source spectra that
  // exist; false where a tile holds more than the staging capacity of its height
  auto compact_tiles = [&](const std::vector<NearTile<D>>& in, int cap, std::vector<NearCTile<D>>& out) {
    for (const NearTile<D>& t : in) {
      NearCTile<D> c{};
      std::memcpy(c.tgt, t.tgt, sizeof c.tgt);
      for (int e = 0; e < kCTileCapMax; ++e) c.src[e] = t.zero;
      for (int j = 0; j < kTileSrcRowsMax * (kTileW + 2); ++j) c.loff[j] = (uint32_t)(cap * 64);
      int n = 0;
      for (int j = 0; j < 4 * (t.rz + 2) * (kTileW + 2); ++j) {
        if (t.src[j] == t.zero) continue;
        if (n == cap) return false;
        c.src[n] = t.src[j];
        c.loff[j] = (uint32_t)(n * 64);
        const int x = j % (kTileW + 2);
        if (x == 0 || x == kTileW + 1) c.edges = 1;
        ++n;
      }
      c.src_mask = t.src_mask;
      c.row_mask = t.row_mask;
      c.nreal = n;
      c.rz = t.rz;
      c.zero = t.zero;
      c.fhat = t.fhat;
      c.uhat = t.uhat;
      c.kptr = t.kptr;
      out.push_back(c);
    }
    return !out.empty();
  };
  auto JW = [&](int64_t blk) { return (double*)p->jw + blk * N3; };
  auto WW = [&](int64_t blk) { return (double*)p->w + blk * N3; };

  HostItems hi;
  std::vector<PendingStep> steps, rsteps, alt_steps;
  PendingStep corr_conv{};                       // the correction pass's base-level convert
  std::vector<size_t> alt_of;                    // primary step index of each alternative
  // chain: 0 before the level's fork, 1 base-level super-block path, 2 far field, 3 after the
  // join (see run_steps); -1 derives it from the phase
  auto push = [&](std::vector<PendingStep>& dst, int l, int phase, int sub, int kind, int ty, size_t off,
                  size_t count, const double* wt, int64_t work = 0, int mode = 0, int chain = -1) {
    if (chain < 0)
      chain = phase <= 1 ? 0 : (phase >= 7 || (kind == K_INTERP && sub == 100)) ? 3 : 2;
    if (count) dst.push_back({l, phase, sub, kind, ty, off, (int32_t)count, wt, work, mode, chain});
  };

  // coarsening (before level 0), bottom-up over levels
  for (int l = LR - 2; l >= 0; --l) {
    std::vector<CoarsenItem> it;
    for (int i : ids[l]) {
      if (leaf[i]) continue;
      CoarsenItem c{};
      c.dst = p->fe + i * N3;
      for (int oc = 0; oc < 8; ++oc) {
        const int ch = child_of(i, oc);
        c.child[oc] = leaf[ch] ? nullptr : p->fe + ch * N3;
        c.child_in[oc] = ch * N3;
      }
      it.push_back(c);
    }
    push(steps, 0, 0, LR - 2 - l, K_COARSEN, TY_F64, hi.add(it), it.size(), nullptr);
  }

  // An FP64 plan on a single-level layout reads its base-level sources straight from the pass's
  // input in the super-block transforms and the first anterpolation, so its convert pass (a
  // copy) is dropped.  FP32 plans keep the FP32 copy: the anterpolation reads each child block
  // once per parent slab, and FP64 children there cost more than the convert saves.
  const bool direct_in = p->super_base && LR == 1 && tyb == TY_F64 && !p->correction;
  std::vector<int64_t> block_of_src(nsrc[tyb], -1);    // base source slot -> block index
  for (int i : ids[0]) block_of_src[base_src_slot[i]] = i;
  for (int l = 0; l < LR; ++l) {
    const double h = std::ldexp(1.0, -l);
    if (l == 0 && !direct_in) {
      std::vector<ConvertItem<D>> it;
      for (int i : ids[0]) {
        ConvertItem<D> c{};
        c.dst = SRC(tyb, base_src_slot[i]);
        c.src = leaf[i] ? nullptr : p->fe + i * N3;
        c.src_in = i * N3;
        it.push_back(c);
      }
      push(steps, l, 1, 0, K_CONVERT, tyb, hi.add(it), it.size(), nullptr);
    } else if (l > 0) {
      std::vector<RefineItem> rit;
      std::vector<CorrectItem<D>> cit;
      for (int i : ids[l]) {
        const I3 c = coords[i];
        const int par = cmap[l - 1].at(parent_of(c));
        RefineItem r{};
        r.jw = JW(i);
        r.parent_w = WW(par);
        r.octant = octant_of(c);
        rit.push_back(r);
        CorrectItem<D> q{};
        q.g = SRC(tyb, base_src_slot[i]);
        q.f = leaf[i] ? nullptr : p->fe + i * N3;
        q.f_in = i * N3;
        q.jw = JW(i);
        for (int face = 0; face < 6; ++face) {
          const int nbi = face_nbr(i, face);
          q.nbr[face] = nbi >= 0 ? JW(nbi) : nullptr;
        }
        q.parent_w = WW(par);
        q.octant = octant_of(c);
        q.inv_h2 = 1.0 / (h * h);
        cit.push_back(q);
      }
      push(steps, l, 1, 0, K_REFINE, TY_F64, hi.add(rit), rit.size(), p->d_w3);
      push(steps, l, 1, 1, K_CORRECT, tyb, hi.add(cit), cit.size(), p->d_w3);
    }
    const int K = (int)chT[l].lv.size();
    std::vector<std::vector<AnterpItem<D, D>>> ant(K);
    std::vector<std::vector<InterpItem<D, D>>> itp(K);
    std::vector<FftFwdItem<D>> fwd[2];
    std::vector<FftInvItem<D>> inv[2];
    std::vector<std::vector<MacTile<D>>> rows(K);      // per octree level (one kernel set each)
    std::vector<int64_t> work(K, 0);
    // row width of each octree level's tiles: 4 targets where rows of 8 would be mostly empty
    // (levels a few blocks wide).  Cost per wavefront and source row: the W + 6 source and 7
    // kernel spectra it loads plus its W target accumulations.
    std::vector<int> wsel(K, kMacL);
    {
      std::vector<double> cost[2] = {std::vector<double>(K, 0.0), std::vector<double>(K, 0.0)};
      for (int ch = 0; ch < 2; ++ch) {
        if (ch == 1 && !hasA[l]) continue;
        for (const TileDesc& rd : (ch == 0 ? chT[l] : chA[l]).rows) {
          int active = 0;
          for (int q = 0; q < 4; ++q)
            for (int i = 0; i < rd.W; ++i)
              if (rd.tgt_node[q][i] >= 0) {
                ++active;
                break;
              }
          cost[rd.W == kMacL ? 0 : 1][rd.k] +=
              (double)active * __builtin_popcountll(rd.mask) * (2 * rd.W + 13);
        }
      }
      for (int k = 0; k < K; ++k)
        if (cost[1][k] < cost[0][k]) wsel[k] = kMacL / 2;
    }
    std::vector<std::vector<MacTile<D>>> alt_mac(K);   // the other width, for the autotuner
    std::vector<char> fwd_done[2] = {std::vector<char>(nsrc[0], 0), std::vector<char>(nsrc[1], 0)};
    for (int ch = 0; ch < 2; ++ch) {
      if (ch == 1 && !hasA[l]) continue;
      Fmm& F = ch == 0 ? chT[l] : chA[l];
      p->interactions += F.interactions;
      for (size_t k = 0; k < F.level_interactions.size(); ++k) work[k] += F.level_interactions[k];
      for (int k = 1; k < (int)F.lv.size(); ++k) {
        OctLevel& L = F.lv[k];
        OctLevel& C = F.lv[k - 1];
        const int tp = ty_of(k), tc = ty_of(k - 1);
        std::vector<AnterpItem<D, D>> tmpi(L.nodes.size());
        for (size_t i = 0; i < L.nodes.size(); ++i) {
          tmpi[i].dst = L.need_src[i] ? SRC(tp, L.src_slot[i]) : nullptr;
          for (int oc = 0; oc < 8; ++oc) {
            tmpi[i].child[oc] = nullptr;
            tmpi[i].child_in[oc] = -1;
          }
        }
        for (size_t c = 0; c < C.nodes.size(); ++c) {
          const int pi = C.parent[c];
          if (!L.need_src[pi] || !C.is_src[c]) continue;
          if (k == 1 && direct_in)
            tmpi[pi].child_in[octant_of(C.nodes[c])] = block_of_src[C.src_slot[c]] * N3;
          else
            tmpi[pi].child[octant_of(C.nodes[c])] = SRC(tc, C.src_slot[c]);
        }
        for (size_t i = 0; i < L.nodes.size(); ++i)
          if (L.need_src[i]) ant[k].push_back(tmpi[i]);
      }
      for (size_t k = 0; k < F.lv.size(); ++k) {
        OctLevel& L = F.lv[k];
        const int ty = ty_of((int)k);
        const bool blockwise = !(k == 0 && p->super_base);
        for (size_t i = 0; i < L.nodes.size(); ++i) {
          if (blockwise && L.referenced[i] && !fwd_done[ty][L.src_slot[i]]) {
            fwd_done[ty][L.src_slot[i]] = 1;
            fwd[ty].push_back({SRC(ty, L.src_slot[i]), FH(ty, L.src_slot[i])});
          }
          if (blockwise && L.has_ifft[i]) inv[ty].push_back({UH(ty, L.tgt_slot[i]), V(ty, L.tgt_slot[i])});
          if (k + 1 < F.lv.size() && L.has_val[i] && F.lv[k + 1].has_val[L.parent[i]]) {
            InterpItem<D, D> q{};
            q.child = V(ty, L.tgt_slot[i]);
            q.parent = V(ty_of((int)k + 1), F.lv[k + 1].tgt_slot[L.parent[i]]);
            q.octant = octant_of(L.nodes[i]);
            q.accumulate = L.has_ifft[i];
            if (k == 0 && farA && L.has_ifft[i]) {
              q.child = FAR(L.tgt_slot[i]);
              q.accumulate = 0;
              far_used[L.tgt_slot[i]] = 1;
            }
            itp[k].push_back(q);
          }
        }
      }
      for (const TileDesc& rd : F.rows) {
        if (rd.k == 0 && p->super_base) continue;
        if (rd.W != wsel[rd.k] && !p->tune) continue;
        const SpecSet* ss = nullptr;
        LGF_HIP_CHECK(plan_spectra(p, nb, 1 << rd.k, &ss));
        OctLevel& L = F.lv[rd.k];
        const int ty = ty_of(rd.k);
        MacTile<D> m{};
        m.row_mask = 0;
        for (int q = 0; q < 4; ++q)
          for (int i = 0; i < kMacL; ++i) {
            const int t = rd.tgt_node[q][i];
            m.tgt[q][i] = (t >= 0 && L.has_ifft[t]) ? L.tgt_slot[t] : -1;
            if (m.tgt[q][i] >= 0) m.row_mask |= 1 << q;
          }
        for (int j = 0; j < 36; ++j)
          for (int q = 0; q < kMacSlots; ++q) {
            // a node with no source slot (absent, or a source no target here pairs with) reads
            // the all-zero spectrum
            const int id = rd.src_node[j][q];
            const int sl = id >= 0 ? L.src_slot[id] : -1;
            m.src[j][q] = sl >= 0 ? sl : (int)nsrc[ty];
          }
        m.pair_mask = rd.mask;
        m.flags = rd.k == 0 ? 1 : 0;
        m.fhat = FH(ty, 0);
        m.uhat = UH(ty, 0);
        m.kptr = ty == TY_F32 ? (const cpx<D>* const*)ss->kp32 : (const cpx<D>* const*)ss->kp64;
        (rd.W == wsel[rd.k] ? rows : alt_mac)[rd.k].push_back(m);
      }
    }
    for (int ty = 0; ty < 2; ++ty) {
      p->n_fwd += (int64_t)fwd[ty].size();
      p->n_inv += (int64_t)inv[ty].size();
      push(steps, l, 3, 0, K_FWD, ty, hi.add(fwd[ty]), fwd[ty].size(), nullptr, (int64_t)fwd[ty].size());
      push(steps, l, 5, 0, K_INV, ty, hi.add(inv[ty]), inv[ty].size(), nullptr, (int64_t)inv[ty].size());
    }
    for (int k = 0; k < K; ++k) {
      p->n_rows += (int64_t)rows[k].size();
      const int half = wsel[k] == kMacL ? 0 : kMacHalfRows;
      // the shared-source form on coarse levels (and FP64 everywhere); FP32 per-block base
      // levels stage the kernel spectra in LDS.  A coarse level of rows of 4 whose source slots
      // lie within kMacLdsSrc of each other (small levels) takes the LDS form (kernel and source
      // spectra of a frequency chunk staged once per workgroup).
      int shape = (ty_of(k) == TY_F64 || k > 0) ? kMacDefault64 : 0;
      bool lds = false;
      if (half && k > 0 && !rows[k].empty()) {
        const int zero = (int)nsrc[ty_of(k)];
        int lo = std::numeric_limits<int>::max(), hi_s = -1;
        for (const MacTile<D>& m : rows[k])
          for (int j = 0; j < 36; ++j)
            for (int q = 0; q < kMacSlots; ++q)
              if (m.src[j][q] != zero) {
                lo = std::min(lo, m.src[j][q]);
                hi_s = std::max(hi_s, m.src[j][q]);
              }
        if (hi_s >= 0 && hi_s - lo < kMacLdsSrc) {
          for (MacTile<D>& m : rows[k]) {
            m.src_lo = lo;
            m.src_n = hi_s - lo + 1;
            // rows of kMacL / 2: window slot q holds x0 - 3 + q, the targets x0 .. x0 + 3
            bool inner = true;
            for (int j = 0; j < 36; ++j)
              for (int q = 0; q < kMacL / 2 + 6; ++q)
                if ((q < 3 || q >= 3 + kMacL / 2) && m.src[j][q] != zero) inner = false;
            if (inner) m.flags |= 2;
            p->n_lds_inner += inner;
          }
          p->n_lds_tiles += (int64_t)rows[k].size();
          lds = true;
          shape = kMacLds;
        }
      }
      const size_t primary = steps.size();
      push(steps, l, 4, k, K_MAC, ty_of(k), hi.add(rows[k]), rows[k].size(), nullptr, work[k], half | shape);
      if (steps.size() > primary) steps.back().lds = lds;
      if (steps.size() > primary && !alt_mac[k].empty()) {
        push(alt_steps, l, 4, k, K_MAC, ty_of(k), hi.add(alt_mac[k]), alt_mac[k].size(), nullptr, work[k],
             (kMacHalfRows - half) | (lds ? kMacDefault64 : shape));
        alt_of.push_back(primary);
      }
    }
    if (p->super_base) {
      // super-block transforms, near rows and inverse transforms of the base octree level
      for (int k = 0; k < 1; ++k) {
        const int a = arena_of(k), sty = sup_ty(k);
        const int chain = k == 0 ? 1 : 2;
        std::vector<SuperFwdItem<D>> sf;
        for (size_t q = 0; q < sup_src[a].size(); ++q) {
          const SupSrc& ss = sup_src[a][q];
          if (ss.l != l || ss.k != k) continue;
          SuperFwdItem<D> it{};
          for (int oc = 0; oc < 8; ++oc) {
            const int sl = ss.children[oc];
            it.child[oc] = sl >= 0 && !direct_in ? SRC(ty_of(k), sl) : nullptr;
            it.child_in[oc] = sl >= 0 && direct_in ? block_of_src[sl] * N3 : -1;
          }
          it.dst = SFH(a, (int64_t)q);
          it.tmp = it.dst;                 // the z pass transforms the plane stack in place
          sf.push_back(it);
        }
        const SpecSet* ns = nullptr;
        LGF_HIP_CHECK(plan_spectra(p, nb, -(1 << k), &ns));     // super-block kernels, scale 2^k
        std::vector<NearRow<D>> nr;
        std::vector<NearTile<D>> nt, nt4;
        std::vector<SuperInvItem<D>> si_items;
        int64_t pairs = 0;
        const bool tiled = sty == TY_F32;      // FP32 storage: 2 x 2 rows of 4 share staged sources
        for (const SupInst& si : sup) {
          if (si.l != l || si.k != k) continue;
          pairs += si.pairs;
          std::vector<std::pair<I3, int>> tg;
          for (const SupTgt& t : si.tg) tg.push_back({t.c, t.slot});
          if (tiled) {
            make_tiles(tg, si.sslot, (int)nsup_src[a], SFH(a, 0), SUH(a, 0),
                       (const cpx<D>* const*)ns->kp32, nt);
            make_tiles(tg, si.sslot, (int)nsup_src[a], SFH(a, 0), SUH(a, 0),
                       (const cpx<D>* const*)ns->kp32, nt4, 4);
          } else
            make_rows(tg, si.sslot, (int)nsup_src[a], 4, SFH(a, 0), SUH(a, 0), ns->kp64, nr);
          const OctLevel& L = (si.ch == 0 ? chT[l] : chA[l]).lv[k];
          for (const SupTgt& t : si.tg) {
            SuperInvItem<D> v{};
            v.src = SUH(a, t.slot);
            v.tmp = SUH(a, t.slot);          // the z pass transforms the spectrum in place
            for (int oc = 0; oc < 8; ++oc)
              v.child[oc] = t.child[oc] >= 0 ? V(ty_of(k), L.tgt_slot[t.child[oc]]) : nullptr;
            si_items.push_back(v);
          }
        }
        p->n_sup_fwd += (int64_t)sf.size();
        p->n_sup_inv += (int64_t)si_items.size();
        p->n_near_rows += (int64_t)(tiled ? 4 * nt.size() : nr.size());
        p->near_pairs += pairs;
        push(steps, l, 3, k, K_SUP_FWD, sty, hi.add(sf), sf.size(), nullptr, (int64_t)sf.size(), 0, chain);
        const size_t primary = steps.size();
        // tiles of 2 x 4 rows (fewer staged spectra per row, more LDS) where they are about as
        // full as tiles of 2 x 2 (dense levels); the other height is an autotuner candidate
        const bool tall = tiled && 8 * nt4.size() <= 9 * nt.size() / 2;
        if (tall) std::swap(nt, nt4);
        // compact tiles (only the source super-blocks that exist staged), 2 x 4 rows first.
        // FP64 spectra: the fused form where every tile fits (z transforms, MAC and inverse z
        // transforms per line in one kernel: the spectra never go through HBM; FP64 solve of
        // the 8^3 layout of 16^3 blocks 0.31 -> 0.27 ms), else rows.  FP32 spectra: the pipelined near MAC
        // on the same compact tiles (the fused form ties with it there), else the one-chunk
        // tiles.  The autotuner times each candidate with its level's transforms.
        std::vector<NearCTile<D>> ct[2];           // [0]: 2 x 2 rows, [1]: 2 x 4 rows
        if (!tiled) {
          nt.clear();
          nt4.clear();
          for (const SupInst& si : sup) {
            if (si.l != l || si.k != k) continue;
            std::vector<std::pair<I3, int>> tg;
            for (const SupTgt& t : si.tg) tg.push_back({t.c, t.slot});
            make_tiles(tg, si.sslot, (int)nsup_src[a], SFH(a, 0), SUH(a, 0), (const cpx<D>* const*)ns->kp64, nt, 2);
            make_tiles(tg, si.sslot, (int)nsup_src[a], SFH(a, 0), SUH(a, 0), (const cpx<D>* const*)ns->kp64, nt4, 4);
          }
        }
        for (const std::vector<NearTile<D>>* lst : {&nt, &nt4})
          if (!lst->empty()) {
            const int h = (*lst)[0].rz == 4;
            if (!compact_tiles(*lst, near_ctile_cap(h ? kNearTiled + 7 : kNearTiled + 5), ct[h])) ct[h].clear();
            for (NearCTile<D>& c : ct[h])
              c.ktr = tiled ? (const cpx<D>*)ns->col32 : (const cpx<D>*)ns->col64;
          }
        const int piped = !ct[1].empty() ? 1 : !ct[0].empty() ? 0 : -1;
        // the image holds a height's compact tiles only where a step (or alternative) uses them
        size_t ct_off[2] = {0, 0};
        for (int h = 0; h < 2; ++h)
          if (!ct[h].empty() && (h == piped || p->tune)) ct_off[h] = hi.add(ct[h]);
        if (piped >= 0 && tiled)
          push(steps, l, 4, k, K_NEAR_MAC, sty, ct_off[piped], ct[piped].size(), nullptr, pairs,
               piped ? kNearTiled + 7 : kNearTiled + 5, chain);
        else if (piped >= 0)
          push(steps, l, 4, k, K_NEAR_MAC, sty, ct_off[piped], ct[piped].size(), nullptr, pairs,
               kNearFused + (piped ? 4 : 2), chain);
        else if (tiled)
          push(steps, l, 4, k, K_NEAR_MAC, sty, hi.add(nt), nt.size(), nullptr, pairs,
               tall ? kNearTiled + 6 : kNearTiled + 4, chain);
        else {
          push(steps, l, 4, k, K_NEAR_MAC, sty, hi.add(nr), nr.size(), nullptr, pairs, 4, chain);
        }
        const int prim_mode = steps.size() > primary ? steps.back().mode : -1;
        if (p->tune && steps.size() > primary) {
          // the other launch shapes for the autotuner: the compact tiles of both heights in the
          // fused and the pipelined form, the one-chunk tiles (FP32), rows of 2, 4 or 8 targets
          for (int h = 0; h < 2; ++h) {
            if (ct[h].empty()) continue;
            for (int mode : {kNearFused + (h ? 4 : 2), h ? kNearTiled + 7 : kNearTiled + 5}) {
              if (mode == prim_mode) continue;
              push(alt_steps, l, 4, k, K_NEAR_MAC, sty, ct_off[h], ct[h].size(), nullptr, pairs, mode, chain);
              alt_of.push_back(primary);
            }
          }
          if (tiled)
            for (const std::vector<NearTile<D>>* lst : {&nt, &nt4}) {
              if (lst->empty()) continue;
              const int mode = (*lst)[0].rz == 4 ? kNearTiled + 6 : kNearTiled + 4;
              if (mode == prim_mode) continue;
              push(alt_steps, l, 4, k, K_NEAR_MAC, sty, hi.add(*lst), lst->size(), nullptr, pairs, mode, chain);
              alt_of.push_back(primary);
            }
          for (int shape : {2, 4, 8}) {        // rows of 2 suit sparse levels
            if (shape == prim_mode) continue;
            std::vector<NearRow<D>> alt_rows;
            for (const SupInst& si : sup) {
              if (si.l != l || si.k != k) continue;
              std::vector<std::pair<I3, int>> tg;
              for (const SupTgt& t : si.tg) tg.push_back({t.c, t.slot});
              make_rows(tg, si.sslot, (int)nsup_src[a], shape, SFH(a, 0), SUH(a, 0), ns->kp64, alt_rows);
            }
            push(alt_steps, l, 4, k, K_NEAR_MAC, sty, hi.add(alt_rows), alt_rows.size(), nullptr, pairs, shape,
                 chain);
            alt_of.push_back(primary);
          }
        }
        push(steps, l, 5, k, K_SUP_INV, sty, hi.add(si_items), si_items.size(), nullptr,
             (int64_t)si_items.size(), 0, chain);
      }
    }
    for (int k = 1; k < K; ++k) {
      const int ty = (k == 1 && direct_in) ? TY_F64
                     : (ty_of(k - 1) == TY_F32 && ty_of(k) == TY_F64) ? TY_MIX : ty_of(k);
      push(steps, l, 2, k, K_ANTERP, ty, hi.add(ant[k]), ant[k].size(), p->d_w);
    }
    for (int k = K - 2; k >= 0; --k) {
      const int ty = (ty_of(k) == TY_F32 && ty_of(k + 1) == TY_F64) ? TY_MIX : ty_of(k);
      push(steps, l, 6, 100 - k, K_INTERP, ty, hi.add(itp[k]), itp[k].size(), p->d_w, 0, 0,
           k == 0 && farA ? 2 : -1);
    }
    std::vector<CombineItem<D>> cmb;
    const double h2 = h * h;
    for (size_t a = 0; a < ids[l].size(); ++a) {
      const int i = ids[l][a];
      CombineItem<D> c{};
      c.dst_out = i * N3;
      const int ts = chT[l].lv[0].tgt_slot[a];
      c.v = ts >= 0 ? V(tyb, ts) : nullptr;
      c.far = ts >= 0 && far_used[ts] ? FAR(ts) : nullptr;
      c.base = l > 0 ? JW(i) : nullptr;
      c.scale = h2;
      cmb.push_back(c);
      if (!leaf[i]) {
        CombineItem<D> q{};
        q.dst_d = WW(i);
        const int ta = chA[l].lv[0].tgt_slot[a];
        q.v = ta >= 0 ? V(tyb, ta) : nullptr;
        q.far = ta >= 0 && far_used[ta] ? FAR(ta) : nullptr;
        q.base = l > 0 ? JW(i) : nullptr;
        q.scale = h2;
        cmb.push_back(q);
      }
    }
    push(steps, l, 7, 0, K_COMBINE, tyb, hi.add(cmb), cmb.size(), nullptr);
  }

  p->base_slot = base_src_slot;
  if (p->correction) {
    // run as a correction pass, this plan's base-level leaf sources are written by the
    // residual in FP32: its convert then only handles the coarsened non-leaf blocks
    std::vector<ConvertItem<D>> cc;
    for (int64_t i = 0; i < n; ++i)
      if (lev[i] == 0 && !leaf[i]) {
        ConvertItem<D> c{};
        c.dst = SRC(tyb, base_src_slot[i]);
        c.src = p->fe + i * N3;
        cc.push_back(c);
      }
    corr_conv = {0, 1, 0, K_CONVERT, tyb, hi.add(cc), (int32_t)cc.size(), nullptr, 0, 0, 0};
  }
  if (p->fp32 && p->dc_iters > 0) {
    // r = f - L u: in FP32 straight into the correction plan's base-level leaf sources, in FP64
    // for the blocks of finer levels, which the correction pass coarsens and corrects
    const Plan* q = p->corr;
    std::vector<ResidualItem> it;
    for (int64_t i = 0; i < n; ++i) {
      ResidualItem r{};
      r.r = lev[i] > 0 ? p->r + i * N3 : nullptr;
      r.conv = lev[i] == 0 && leaf[i] ? (float*)q->src + (int64_t)q->base_slot[i] * N3 : nullptr;
      r.off = i * N3;
      for (int face = 0; face < 6; ++face) {
        const int nbi = face_nbr((int)i, face);
        r.nbr_off[face] = nbi >= 0 ? (int64_t)nbi * N3 : -1;
      }
      const double h = std::ldexp(1.0, -lev[i]);
      r.inv_h2 = 1.0 / (h * h);
      r.leaf = leaf[i];
      it.push_back(r);
    }
    push(rsteps, 0, 0, 0, K_RESIDUAL, TY_F64, hi.add(it), it.size(), nullptr);
  }

  // every item must stay inside the plan's device ranges before anything is launched
  {
    SlotCounts sc{{nsrc[0], nsrc[1]}, {ntgt[0], ntgt[1]}, {nsup_src[0], nsup_src[1]},
                  {nsup_tgt[0], nsup_tgt[1]}};
    std::set<uint32_t> rel;
    const uint8_t* img = hi.buf.data();
    for (const auto* list : {&steps, &rsteps, &alt_steps})
      for (const PendingStep& st : *list)
        if (!validate_step(p, st.kind, st.ty, st.mode, img + st.off, st.count, n, sc, err, img, &rel))
          return hipErrorInvalidValue;
    if (corr_conv.count &&
        !validate_step(p, corr_conv.kind, corr_conv.ty, 0, img + corr_conv.off, corr_conv.count, n, sc, err, img, &rel))
      return hipErrorInvalidValue;
    // every word of the image that carries the workspace tag must be a pointer field the checks
    // above recorded (else relocation would miss it, or the tag would hit a non-pointer)
    hi.buf.resize((hi.buf.size() + 7) / 8 * 8);
    int64_t tagged = 0;
    for (size_t w = 0; w < hi.buf.size() / 8; ++w) {
      uint64_t v;
      std::memcpy(&v, hi.buf.data() + 8 * w, 8);
      if ((v >> kVTagShift) != (kVBase >> kVTagShift)) continue;
      ++tagged;
      if (!rel.count((uint32_t)w) || v - kVBase >= (uint64_t)p->vnext) {
        if (err) *err = "internal: item word " + std::to_string(w) + " holds an unrecorded workspace address";
        return hipErrorInvalidValue;
      }
    }
    if (tagged != (int64_t)rel.size() || hi.buf.size() / 8 >= ((size_t)1 << 32)) {
      if (err) *err = "internal: relocation table does not match the item image";
      return hipErrorInvalidValue;
    }
    p->relocs.assign(rel.begin(), rel.end());
  }
  p->h_items = hi.buf;
  LGF_HIP_CHECK(ar.alloc(&p->d_items, hi.buf.size()));
  if (!hi.buf.empty() && !p->dry)
    LGF_HIP_CHECK(hipMemcpy(p->d_items, hi.buf.data(), hi.buf.size(), hipMemcpyHostToDevice));
  {
    void* d = nullptr;
    LGF_HIP_CHECK(ar.alloc(&d, p->relocs.size() * sizeof(uint32_t)));
    p->d_relocs = (uint32_t*)d;
    if (!p->relocs.empty() && !p->dry)
      LGF_HIP_CHECK(hipMemcpy(p->d_relocs, p->relocs.data(), p->relocs.size() * sizeof(uint32_t),
                              hipMemcpyHostToDevice));
  }
  {
    // block table of the forward operators (every plan, every block)
    std::vector<OpItem> ops(n);
    for (int64_t i = 0; i < n; ++i) {
      OpItem& o = ops[i];
      o.off = i * N3;
      for (int face = 0; face < 6; ++face) {
        const int nbi = face_nbr((int)i, face);
        o.nbr_off[face] = nbi >= 0 ? (int64_t)nbi * N3 : -1;
      }
      o.inv_h = std::ldexp(1.0, lev[i]);
      o.leaf = leaf[i];
      o.par_off = lev[i] > 0 ? (int64_t)cmap[lev[i] - 1].at(parent_of(coords[i])) * N3 : -1;
      o.octant = lev[i] > 0 ? octant_of(coords[i]) : 0;
    }
    LGF_HIP_CHECK(ar.alloc(&p->d_ops, ops.size() * sizeof(OpItem)));
    if (n > 0 && !p->dry)
      LGF_HIP_CHECK(hipMemcpy(p->d_ops, ops.data(), ops.size() * sizeof(OpItem), hipMemcpyHostToDevice));
  }
  auto fin = [&](const std::vector<PendingStep>& in, std::vector<Step>& out) {
    for (const PendingStep& s : in)
      out.push_back({s.l, s.phase, s.sub, s.kind, s.ty, (int64_t)s.off, s.count, s.w, s.work, s.mode, s.chain, s.lds});
  };
  fin(steps, p->pass);
  fin(rsteps, p->residual);
  sync_super_modes(p);
  if (p->correction) {
    for (size_t i = 0; i < p->pass.size(); ++i)
      if (p->pass[i].kind == K_CONVERT && p->pass[i].l == 0) p->conv_idx = (int64_t)i;
    std::vector<Step> cv;
    fin({corr_conv}, cv);
    p->conv_corr = cv[0];
  }
  {
    std::vector<Step> alts;
    fin(alt_steps, alts);
    for (size_t i = 0; i < alts.size(); ++i) p->alt.push_back({alt_of[i], alts[i]});
  }
  std::set<int> used;
  for (int l = 0; l < LR; ++l)
    for (const TileDesc& rd : chT[l].rows) used.insert(rd.k);
  // spectra referenced: per octree level with interactions, the 27 super-block kernels at the
  // base level, or the block kernels of the lists
  p->n_spectra = 0;
  for (int k : used) p->n_spectra += k == 0 ? (p->super_base ? 27 : 343) : 316;
  (void)err;
  return hipSuccess;
}

}  // namespace

hipError_t plan_autotune(Plan* p, Binding* b, hipStream_t st);

// The super-block transforms of a level follow its near step: line-major planes (mode 1) for the
// fused form, the plane stack and spectra (mode 0) for every other form.
void sync_super_modes(Plan* p) {
  std::map<std::pair<int, int>, int> lm;
  for (const Step& s : p->pass)
    if (s.kind == K_NEAR_MAC) lm[{s.l, s.sub}] = near_fused(s.mode) ? 1 : 0;
  for (Step& s : p->pass)
    if (s.kind == K_SUP_FWD || s.kind == K_SUP_INV) {
      auto it = lm.find({s.l, s.sub});
      s.mode = it != lm.end() ? it->second : 0;
    }
}

hipError_t plan_build(const int32_t* blocks, const int32_t* levels, int64_t n, int nb, int n_i,
                      bool fp32, int dc_iters, uint64_t budget, Plan** out, std::string* err, bool dry,
                      bool autotune, bool super_base) {
  Plan* p = new Plan();
  p->super_base = super_base;
  p->tune = autotune;
  p->nb = nb;
  p->n_i = n_i;
  p->fp32 = fp32;
  p->dc_iters = fp32 ? dc_iters : 0;
  p->nblocks = n;
  p->dry = dry;
  hipError_t e = dry ? hipSuccess : device_ctx(&p->ctx);
  if (e != hipSuccess) {
    delete p;
    return e;
  }
  std::vector<I3> coords(n);
  std::vector<int> lev(n);
  int LR = 0;
  for (int64_t i = 0; i < n; ++i) {
    coords[i] = {blocks[3 * i], blocks[3 * i + 1], blocks[3 * i + 2]};
    lev[i] = levels ? levels[i] : 0;
    LR = std::max(LR, lev[i] + 1);
  }
  p->LR = LR;
  if (p->fp32 && p->dc_iters > 0) {
    // the defect-correction re-solve: the same layout, every level and spectrum in FP32
    Plan* q = new Plan();
    q->super_base = super_base;
    q->tune = autotune;
    q->nb = nb;
    q->n_i = n_i;
    q->fp32 = true;
    q->all_fp32 = true;
    q->correction = true;
    q->nblocks = n;
    q->dry = dry;
    q->ctx = p->ctx;
    q->LR = LR;
    p->corr = q;
    e = build_plan(q, coords, lev, budget, err);
    // the residual writes into the correction plan's buffers; its workspace continues the same
    // virtual range
    p->ranges = q->ranges;
    p->next_fake = q->next_fake;
    p->vnext = q->vnext;
  }
  if (e == hipSuccess) {
    // one HBM budget for both plans (1 byte: already exhausted)
    const uint64_t used = p->corr ? (uint64_t)p->corr->bytes : 0;
    e = build_plan(p, coords, lev, budget == 0 ? 0 : budget > used ? budget - used : 1, err);
  }
  if (e == hipSuccess) {
    // binding layout: [workspace of both plans | main item image | correction item image]
    auto al = [](int64_t v) { return (v + 255) / 256 * 256; };
    p->items_at = al(p->ws_bytes);
    p->bind_bytes = p->items_at + al((int64_t)p->h_items.size());
    if (p->corr) {
      p->corr->items_at = p->bind_bytes;
      p->bind_bytes += al((int64_t)p->corr->h_items.size());
      p->corr->bind_bytes = p->bind_bytes;
    }
    p->budget = budget;
    // a solve needs one binding next to the constants
    const int64_t cst = p->bytes + (p->corr ? p->corr->bytes : 0);
    if (budget && (uint64_t)(cst + p->bind_bytes) > budget) e = hipErrorOutOfMemory;
  }
  if (e == hipSuccess && autotune && !dry) {
    // time the launch shapes on a binding of the plan's own, kept for its first solve
    Binding* b = nullptr;
    e = plan_binding(p, p->ctx->stream, 0, &b);
    if (e == hipSuccess && p->corr) e = plan_autotune(p->corr, b, p->ctx->stream);
    if (e == hipSuccess) e = plan_autotune(p, b, p->ctx->stream);
    if (e == hipSuccess) {
      std::lock_guard<std::mutex> lk(p->bmu);
      p->bindings.erase({p->ctx->stream, 0});
      p->idle.push_back(b);
    }
  }
  if (e != hipSuccess) {
    plan_free(p);
    return e;
  }
  *out = p;
  return hipSuccess;
}

hipError_t plan_set_mac_shape(Plan* p, int shape) {
  if (shape != 0 && shape != 1 && shape != 2 && shape != 4 && shape != 6 && shape != 8 && shape != kMacLds)
    return hipErrorInvalidValue;
  if (p->corr) LGF_HIP_CHECK(plan_set_mac_shape(p->corr, shape));
  if (p->mac_mode0.empty())
    for (const Step& s : p->pass) p->mac_mode0.push_back(s.mode);
  auto has = [](int ty, int m) {
    return ty == TY_F32 ? (m == 1 || m == 2 || m == 4 || m == 8) : (m == 1 || m == 2 || m == 6 || m == 8);
  };
  for (size_t i = 0; i < p->pass.size(); ++i) {
    Step& s = p->pass[i];
    if (s.kind != K_MAC) continue;
    if (shape == 0) s.mode = p->mac_mode0[i];
    else if (shape == kMacLds ? s.lds : has(s.ty, shape)) s.mode = shape | (p->mac_mode0[i] & kMacHalfRows);
  }
  if (!p->dry) graph_forget(p);
  return hipSuccess;
}

hipError_t plan_set_near_shape(Plan* p, int shape) {
  // the correction plan (FP32 spectra) takes the shape where it has it
  if (p->corr) (void)plan_set_near_shape(p->corr, shape);
  if (p->near0.empty()) p->near0 = p->pass;
  std::vector<std::pair<size_t, Step>> pick;
  for (size_t i = 0; i < p->near0.size(); ++i) {
    const Step& s0 = p->near0[i];
    if (s0.kind != K_NEAR_MAC) continue;
    const Step* c = (shape == 0 || s0.mode == shape) ? &s0 : nullptr;
    for (const auto& pa : p->alt)
      if (!c && pa.first == i && pa.second.mode == shape) c = &pa.second;
    if (c) {
      pick.push_back({i, *c});
      continue;
    }
    // the fused and the pipelined form of compact tiles of one height run on the same items
    if (near_compact(s0.mode) && near_compact(shape) && near_ctile_rz(s0.mode) == near_ctile_rz(shape)) {
      Step x = s0;
      x.mode = shape;
      pick.push_back({i, x});
      continue;
    }
    return hipErrorInvalidValue;
  }
  for (const auto& pc : pick) p->pass[pc.first] = pc.second;
  sync_super_modes(p);
  if (!p->dry) graph_forget(p);
  return hipSuccess;
}

void plan_free(Plan* p) {
  if (!p) return;
  plan_free(p->corr);
  if (!p->dry) {
    graph_forget(p);
    // bindings may still be in use by work the caller enqueued
    (void)hipDeviceSynchronize();
    for (auto& kv : p->bindings) p->idle.push_back(kv.second);
    for (Binding* b : p->idle) {
      if (b->owned) (void)hipFree(b->base);
      delete b;
    }
    for (void* a : p->allocs) (void)hipFree(a);
  }
  delete p;
}

// ----------------------------------------------------------------------------- bindings
namespace {
std::atomic<bool> g_poison{false};
}  // namespace

void set_poison(bool on) { g_poison = on; }

hipError_t bind(Plan* p, Binding* b, hipStream_t st, bool force) {
  if (p->dry || !b || !b->base) return hipErrorInvalidValue;
  if (b->bytes < p->bind_bytes) return hipErrorInvalidValue;
  if (b->plan == p && !force && !g_poison) return hipSuccess;
  b->plan = nullptr;
  const uint64_t delta = (uint64_t)(uintptr_t)b->base - kVBase;
  for (Plan* q : {p->corr, p}) {
    if (!q || q->h_items.empty()) continue;
    uint8_t* dst = b->base + q->items_at;
    LGF_HIP_CHECK(hipMemcpyAsync(dst, q->d_items, q->h_items.size(), hipMemcpyDeviceToDevice, st));
    LGF_HIP_CHECK(launch_relocate((uint64_t*)dst, q->d_relocs, (int64_t)q->relocs.size(), delta, st));
  }
  if (g_poison) {
    FillRanges all{};
    all.n = 1;
    all.off[0] = 0;
    all.bytes[0] = p->ws_bytes / 16 * 16;
    LGF_HIP_CHECK(launch_fill(b->base, all, 0xFFFFFFFFu, st));
  }
  FillRanges z{};
  for (Plan* q : {p->corr, p})
    if (q)
      for (const auto& r : q->zero) {
        if (z.n == kFillMax) {
          LGF_HIP_CHECK(launch_fill(b->base, z, 0u, st));
          z.n = 0;
        }
        z.off[z.n] = r.first;
        z.bytes[z.n] = r.second;
        ++z.n;
      }
  LGF_HIP_CHECK(launch_fill(b->base, z, 0u, st));
  b->plan = p;
  return hipSuccess;
}

hipError_t plan_binding(Plan* p, hipStream_t st, int k, Binding** out) {
  std::lock_guard<std::mutex> lk(p->bmu);
  const auto key = std::make_pair(st, k);
  auto it = p->bindings.find(key);
  if (it != p->bindings.end()) {
    *out = it->second;
    return hipSuccess;
  }
  Binding* b = nullptr;
  if (!p->idle.empty()) {
    b = p->idle.back();
    p->idle.pop_back();
  } else {
    const int64_t cst = p->bytes + (p->corr ? p->corr->bytes : 0);
    if (p->budget && (uint64_t)(cst + p->bound_bytes + p->bind_bytes) > p->budget) return hipErrorOutOfMemory;
    void* base = nullptr;
    LGF_HIP_CHECK(hipMalloc(&base, p->bind_bytes));
    b = new Binding{(uint8_t*)base, p->bind_bytes, nullptr, true};
    p->bound_bytes += p->bind_bytes;
  }
  hipError_t e = bind(p, b, st);
  if (e != hipSuccess) {
    p->idle.push_back(b);
    return e;
  }
  p->bindings[key] = b;
  *out = b;
  return hipSuccess;
}

hipError_t plan_trim(Plan* p) {
  std::lock_guard<std::mutex> lk(p->bmu);
  if (p->bindings.empty() && p->idle.empty()) return hipSuccess;
  LGF_HIP_CHECK(hipDeviceSynchronize());
  graph_forget(p);
  for (auto& kv : p->bindings) p->idle.push_back(kv.second);
  p->bindings.clear();
  for (Binding* b : p->idle) {
    if (b->owned) {
      (void)hipFree(b->base);
      p->bound_bytes -= b->bytes;
    }
    delete b;
  }
  p->idle.clear();
  return hipSuccess;
}

// ----------------------------------------------------------------------------- execution
namespace {

template <typename T>
hipError_t launch_kind(int kind, int nb, SetTable& t, hipStream_t st, int mode) {
  switch (kind) {
    case K_CONVERT: return launch_convert<T>(nb, t, st);
    case K_REFINE: return launch_refine(nb, t, st);
    case K_CORRECT: return launch_correct<T>(nb, t, st);
    case K_ANTERP: return launch_anterp<T, T>(nb, t, st);
    case K_FWD: return launch_fft_fwd<T>(nb, t, st);
    case K_MAC: return launch_mac<T>(nb, t, st, mode);
    case K_INV: return launch_fft_inv<T>(nb, t, st);
    case K_INTERP: return launch_interp<T, T>(nb, t, st);
    case K_COMBINE: return launch_combine<T>(nb, t, st);
    case K_COARSEN: return launch_coarsen(nb, t, st);
    case K_RESIDUAL: return launch_residual(nb, t, st);
    case K_SUP_FWD: return launch_super_fwd<T, T>(nb, t, st, mode);
    case K_NEAR_MAC: return launch_near_mac<T>(nb, t, st, mode);
    case K_SUP_INV: return launch_super_inv<T, T>(nb, t, st, mode);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_typed(int kind, int ty, int nb, SetTable& t, hipStream_t st, int mode = 0) {
  if (ty == 0) return launch_kind<float>(kind, nb, t, st, mode);
  if (ty == 1) return launch_kind<double>(kind, nb, t, st, mode);
  if (kind == K_ANTERP) return launch_anterp<float, double>(nb, t, st);
  if (kind == K_INTERP) return launch_interp<float, double>(nb, t, st);
  // FP64 super-block spectra of FP32 child blocks
  if (kind == K_SUP_FWD) return launch_super_fwd<double, float>(nb, t, st, mode);
  if (kind == K_SUP_INV) return launch_super_inv<double, float>(nb, t, st, mode);
  if (kind == K_NEAR_MAC) return launch_near_mac<double>(nb, t, st, mode);
  return hipErrorInvalidValue;
}

struct Ref {
  int l, phase, sub, kind, nb, ty, mode;
  int member;
  const Step* step;
  bool operator<(const Ref& o) const {
    if (l != o.l) return l < o.l;
    if (phase != o.phase) return phase < o.phase;
    if (sub != o.sub) return sub < o.sub;
    if (kind != o.kind) return kind < o.kind;
    if (nb != o.nb) return nb < o.nb;
    if (ty != o.ty) return ty < o.ty;
    if (mode != o.mode) return mode < o.mode;
    return member < o.member;
  }
};

}  // namespace

namespace {
struct ProfRec { int kind, ty, nb, mode; int64_t work; hipEvent_t a, b; };
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof;
}  // namespace

void profile_enable(bool on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = on;
}

hipError_t profile_collect(std::vector<ProfileEntry>* out) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  std::map<std::array<int, 4>, ProfileEntry> acc;
  for (ProfRec& r : g_prof) {
    LGF_HIP_CHECK(hipEventSynchronize(r.b));
    float ms = 0.f;
    LGF_HIP_CHECK(hipEventElapsedTime(&ms, r.a, r.b));
    ProfileEntry& e = acc[{r.kind, r.ty, r.nb, r.mode}];
    e.kind = r.kind; e.ty = r.ty; e.nb = r.nb; e.mode = r.mode;
    e.launches += 1;
    e.ms += ms;
    e.work += r.work;
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g_prof.clear();
  out->clear();
  for (auto& kv : acc) out->push_back(kv.second);
  return hipSuccess;
}

// Within a refinement level the base-level super-block path (forward super-block FFTs, near MAC,
// inverse) and the far field (anterpolation, coarse-level FFTs and MACs, interpolation down to
// level 1) depend only on the level's sources and meet at the interpolation into the base
// level.  The far-field kernels are small and latency-bound, so the base path runs on a second
// stream beside them: fork after the level's sources are formed, join before the base-level
// interpolation.  Chains: 0 before the fork, 1 base path (second stream), 2 far field, 3 after.
namespace {
int chain_of(const Ref& r) { return r.step->chain; }

// one second stream per (thread, device), default priority, and a reusable event pool
struct ForkRes {
  std::map<int, hipStream_t> aux;
  std::vector<hipEvent_t> ev;
};
thread_local ForkRes t_fork;

hipError_t fork_stream(hipStream_t* out) {
  int dev = 0;
  LGF_HIP_CHECK(hipGetDevice(&dev));
  auto it = t_fork.aux.find(dev);
  if (it == t_fork.aux.end()) {
    hipStream_t s = nullptr;
    LGF_HIP_CHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    it = t_fork.aux.emplace(dev, s).first;
  }
  *out = it->second;
  return hipSuccess;
}

hipError_t fork_event(size_t i, hipEvent_t* out) {
  while (t_fork.ev.size() <= i) {
    hipEvent_t e = nullptr;
    LGF_HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    t_fork.ev.push_back(e);
  }
  *out = t_fork.ev[i];
  return hipSuccess;
}

// dst waits for all work enqueued on src so far
hipError_t stream_after(hipStream_t dst, hipStream_t src, size_t ev_index) {
  hipEvent_t e = nullptr;
  LGF_HIP_CHECK(fork_event(ev_index, &e));
  LGF_HIP_CHECK(hipEventRecord(e, src));
  return hipStreamWaitEvent(dst, e, 0);
}
}  // namespace

hipError_t run_steps(const std::vector<Member>& m, bool residual, hipStream_t st, bool one_stream) {
  std::vector<Ref> refs;
  for (size_t i = 0; i < m.size(); ++i) {
    const Plan* q = m[i].p;
    const std::vector<Step>& sv = residual ? q->residual : q->pass;
    for (size_t j = 0; j < sv.size(); ++j) {
      const Step* s = &sv[j];
      // a correction pass's base-level leaf sources were written by the residual
      if (!residual && m[i].accumulate && (int64_t)j == q->conv_idx) s = &q->conv_corr;
      if (s->count == 0) continue;
      refs.push_back({s->l, s->phase, s->sub, s->kind, q->nb, s->ty, s->mode, (int)i, s});
    }
  }
  std::sort(refs.begin(), refs.end());
  bool prof;
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    prof = g_prof_on && !one_stream;
  }
  // per-launch timing (and LGF_NO_FORK) keeps one stream, so that kernel times are not shared
  static const bool no_fork = std::getenv("LGF_NO_FORK") != nullptr;
  std::set<int> base_chain;                      // levels with a base-level super-block path
  if (!prof && !no_fork && !one_stream)
    for (const Ref& r : refs)
      if (chain_of(r) == 1) base_chain.insert(r.l);
  hipStream_t aux = nullptr;
  if (!base_chain.empty()) LGF_HIP_CHECK(fork_stream(&aux));
  bool forked = false;
  int fork_l = -1;
  size_t nev = 0;
  size_t a = 0;
  while (a < refs.size()) {
    size_t b = a;
    SetTable t;
    t.n = 0;
    t.pad = 0;
    while (b < refs.size() && t.n < kMaxSets && refs[b].l == refs[a].l && refs[b].phase == refs[a].phase &&
           refs[b].sub == refs[a].sub && refs[b].kind == refs[a].kind && refs[b].nb == refs[a].nb &&
           refs[b].ty == refs[a].ty && refs[b].mode == refs[a].mode) {
      const Member& mm = m[refs[b].member];
      WorkSet& ws = t.s[t.n++];
      ws.items = mm.b->base + mm.p->items_at + refs[b].step->items;
      ws.count = refs[b].step->count;
      ws.wg_begin = 0;
      ws.aux = mm.accumulate ? kAuxAccumulate : 0;
      ws.in = mm.in;
      ws.out = mm.out;
      ws.w = refs[b].step->w;
      ++b;
    }
    const int c = chain_of(refs[a]), l = refs[a].l;
    if (forked && (l != fork_l || c == 0 || c == 3)) {
      LGF_HIP_CHECK(stream_after(st, aux, nev++));          // join
      forked = false;
    }
    if (!forked && (c == 1 || c == 2) && base_chain.count(l)) {
      LGF_HIP_CHECK(stream_after(aux, st, nev++));          // fork
      forked = true;
      fork_l = l;
    }
    hipStream_t ls = (forked && c == 1) ? aux : st;
    ProfRec rec{refs[a].kind, refs[a].ty, refs[a].nb, refs[a].mode, 0, nullptr, nullptr};
    if (prof) {
      for (size_t q = a; q < b; ++q) rec.work += refs[q].step->work;
      LGF_HIP_CHECK(hipEventCreate(&rec.a));
      LGF_HIP_CHECK(hipEventCreate(&rec.b));
      LGF_HIP_CHECK(hipEventRecord(rec.a, ls));
    }
    hipError_t e = launch_typed(refs[a].kind, refs[a].ty, refs[a].nb, t, ls, refs[a].mode);
    if (e != hipSuccess) return e;
    if (prof) {
      LGF_HIP_CHECK(hipEventRecord(rec.b, ls));
      std::lock_guard<std::mutex> lk(g_prof_mu);
      g_prof.push_back(rec);
    }
    a = b;
  }
  if (forked) LGF_HIP_CHECK(stream_after(st, aux, nev++));
  return hipSuccess;
}

hipError_t solve_members(const std::vector<Member>& m, hipStream_t st, bool one_stream) {
  for (const Member& x : m)
    if (!x.b || x.b->plan != x.p) return hipErrorInvalidValue;     // not bound to the plan
  LGF_HIP_CHECK(run_steps(m, false, st, one_stream));
  int iters = 0;
  for (const Member& x : m) iters = std::max(iters, x.p->dc_iters);
  for (int it = 0; it < iters; ++it) {
    std::vector<Member> act, corr;
    for (const Member& x : m)
      if (x.p->dc_iters > it) {
        act.push_back(x);
        // the correction pass reads r (finer levels) from the binding; the residual writes its
        // base-level leaf sources there directly
        corr.push_back({x.p->corr, x.p->r ? (const double*)in_binding(x.b, x.p->r) : nullptr, x.out, true, x.b});
      }
    LGF_HIP_CHECK(run_steps(act, true, st, one_stream));      // r = f - L u
    LGF_HIP_CHECK(run_steps(corr, false, st, one_stream));    // u += S(r): the pass's final combine adds into u
  }
  return hipSuccess;
}

// ----------------------------------------------------------------------------- graphs
namespace {
struct GraphKey {
  std::vector<std::tuple<Plan*, Binding*, const double*, double*>> m;
  bool operator<(const GraphKey& o) const { return m < o.m; }
};
std::mutex g_graph_mu;
std::map<GraphKey, hipGraphExec_t> g_graphs;
constexpr size_t kMaxGraphs = 64;

bool graphs_enabled() {
  static const bool on = std::getenv("LGF_NO_GRAPH") == nullptr;
  return on;
}
}  // namespace

void graph_forget(Plan* p) {
  std::lock_guard<std::mutex> lk(g_graph_mu);
  for (auto it = g_graphs.begin(); it != g_graphs.end();) {
    bool hit = false;
    for (auto& t : it->first.m) hit |= std::get<0>(t) == p;
    if (hit) {
      (void)hipGraphExecDestroy(it->second);
      it = g_graphs.erase(it);
    } else {
      ++it;
    }
  }
}

hipError_t solve_members_graph(const std::vector<Member>& m, hipStream_t st) {
  bool prof;
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    prof = g_prof_on;
  }
  if (!st || prof || !graphs_enabled()) return solve_members(m, st);
  GraphKey key;
  for (const Member& x : m) key.m.emplace_back(x.p, x.b, x.in, x.out);
  {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    auto it = g_graphs.find(key);
    if (it != g_graphs.end()) return hipGraphLaunch(it->second, st);
  }
  LGF_HIP_CHECK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  hipError_t e = solve_members(m, st);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(st, &g);
  if (e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return e;
  }
  LGF_HIP_CHECK(e2);
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  LGF_HIP_CHECK(e);
  {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    if (g_graphs.size() >= kMaxGraphs) {
      (void)hipGraphExecDestroy(g_graphs.begin()->second);
      g_graphs.erase(g_graphs.begin());
    }
    g_graphs[key] = ex;
  }
  return hipGraphLaunch(ex, st);
}

// ----------------------------------------------------------------------------- autotuner
// Chooses the launch shape of every MAC step of a plan by timing each candidate on the plan's
// own work items (5 repetitions, median): the tile MAC's shapes (rows per wavefront, source-row
// split) and the near MAC's (rows of 4 or 8 targets, 2 x 2-row tiles; the planner builds each
// shape's items).  The choice is remembered per (N_b, element type, tile count or pair count)
// for the process and in the file named by LGF_TUNE_CACHE (one "nb key count mode" line per
// entry).  LGF_TUNE_VERBOSE prints every candidate's time on stderr.
namespace {
std::mutex g_tune_mu;
std::map<std::array<int64_t, 3>, int> g_tune;
bool g_tune_loaded = false;

void tune_load() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = std::getenv("LGF_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  long long a, b, c;
  int mode;
  while (std::fscanf(f, "%lld %lld %lld %d", &a, &b, &c, &mode) == 4) g_tune[{a, b, c}] = mode;
  std::fclose(f);
}
void tune_store(const std::array<int64_t, 3>& k, int mode) {
  g_tune[k] = mode;
  const char* path = std::getenv("LGF_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%lld %lld %lld %d\n", (long long)k[0], (long long)k[1], (long long)k[2], mode);
  std::fclose(f);
}
}  // namespace

constexpr int kTuneReps = 5;             // timed launches per candidate (the median counts)

hipError_t plan_autotune(Plan* p, Binding* bd, hipStream_t st) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  // the candidates run on the plan's items relocated into bd (p or p's correction plan)
  const uint8_t* img = bd->base + p->items_at;
  tune_load();
  static const bool verbose = std::getenv("LGF_TUNE_VERBOSE") != nullptr;   // candidate times on stderr
  hipEvent_t a, b;
  LGF_HIP_CHECK(hipEventCreate(&a));
  LGF_HIP_CHECK(hipEventCreate(&b));
  for (std::vector<Step>* list : {&p->pass}) {
    for (Step& s : *list) {
      if (s.kind != K_MAC) continue;
      const int half = s.mode & kMacHalfRows;
      const std::array<int64_t, 3> key{p->nb, s.ty + (half ? 10 : 0) + (s.lds ? 100 : 0), s.count};
      auto it = g_tune.find(key);
      if (it != g_tune.end()) {
        s.mode = it->second | half;
        continue;
      }
      // the planner's shape first, then the type's other shapes
      std::vector<int> cand{s.mode & (kMacHalfRows - 1)};
      for (int m : (s.ty == 0 ? kMacModes32 : kMacModes64))
        if (std::find(cand.begin(), cand.end(), m) == cand.end() && !(m == 1 && cand[0] == 0)) cand.push_back(m);
      float best = 1e30f;
      int best_mode = 0;
      for (size_t c = 0; c < cand.size(); ++c) {
        float t[kTuneReps];
        for (int rep = 0; rep < kTuneReps; ++rep) {
          SetTable tab;
          tab.n = 1;
          tab.pad = 0;
          tab.s[0] = WorkSet{img + s.items, 0, s.count, 0, nullptr, nullptr, s.w};
          LGF_HIP_CHECK(hipEventRecord(a, st));
          LGF_HIP_CHECK(launch_typed(K_MAC, s.ty, p->nb, tab, st, cand[c] | half));
          LGF_HIP_CHECK(hipEventRecord(b, st));
          LGF_HIP_CHECK(hipEventSynchronize(b));
          LGF_HIP_CHECK(hipEventElapsedTime(&t[rep], a, b));
        }
        std::sort(t, t + kTuneReps);
        if (verbose)
          std::fprintf(stderr, "[lgf tune] mac ty %d count %d mode %d: %.1f us\n", s.ty, s.count, cand[c] | half,
                       1e3f * t[kTuneReps / 2]);
        if (c == 0 || t[kTuneReps / 2] < 0.95f * best) {    // the first candidate is the default shape
          best = t[kTuneReps / 2];
          best_mode = cand[c];
        }
      }
      s.mode = best_mode | half;
      tune_store(key, best_mode);
    }
  }
  // steps with other launch shapes and their own items (near MAC shapes, MAC row widths): time
  // each and keep the fastest in the pass; the replaced step takes the winner's place among the
  // alternatives, so that every shape stays available
  std::map<size_t, std::vector<Step>> groups;
  for (const auto& pa : p->alt) groups[pa.first].push_back(pa.second);
  auto choose = [&](size_t idx, const Step& win) {
    Step& prim = p->pass[idx];
    if (win.mode == prim.mode && win.items == prim.items) return;
    for (auto& pa : p->alt)
      if (pa.first == idx && pa.second.mode == win.mode && pa.second.items == win.items) {
        pa.second = prim;
        break;
      }
    prim = win;
  };
  // A near step is timed with its level's super-block transforms in the mode the candidate
  // needs (the fused form takes over their z passes).  The forward transform of an FP64
  // single-level plan reads the pass input: a zero field stands in for it.
  double* din = nullptr;
  auto sibling = [&](const Step& nr, int kind) -> const Step* {
    for (const Step& x : p->pass)
      if (x.kind == kind && x.l == nr.l && x.sub == nr.sub) return &x;
    return nullptr;
  };
  auto launch_one = [&](const Step& x, int mode) -> hipError_t {
    SetTable tab;
    tab.n = 1;
    tab.pad = 0;
    tab.s[0] = WorkSet{img + x.items, 0, x.count, 0, din, nullptr, x.w};
    return launch_typed(x.kind, x.ty, p->nb, tab, st, mode);
  };
  for (auto& g : groups) {
    const Step prim = p->pass[g.first];
    std::vector<Step> cands{prim};
    for (const Step& x : g.second) cands.push_back(x);
    const Step* sf = prim.kind == K_NEAR_MAC ? sibling(prim, K_SUP_FWD) : nullptr;
    const Step* si = prim.kind == K_NEAR_MAC ? sibling(prim, K_SUP_INV) : nullptr;
    if (sf && !din) {
      LGF_HIP_CHECK(hipMalloc(&din, (size_t)p->nblocks * p->nb * p->nb * p->nb * sizeof(double)));
      LGF_HIP_CHECK(hipMemsetAsync(din, 0, (size_t)p->nblocks * p->nb * p->nb * p->nb * sizeof(double), st));
    }
    const std::array<int64_t, 3> key{p->nb, (prim.kind == K_MAC ? 2000 : 1000) + prim.ty, prim.work};
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      for (const Step& c : cands)
        if (c.mode == it->second) {
          choose(g.first, c);
          break;
        }
      continue;
    }
    float best = 1e30f;
    size_t best_i = 0;
    for (size_t c = 0; c < cands.size(); ++c) {
      float t[kTuneReps];
      const int lm = near_fused(cands[c].mode) ? 1 : 0;
      for (int rep = 0; rep < kTuneReps; ++rep) {
        LGF_HIP_CHECK(hipEventRecord(a, st));
        if (sf) LGF_HIP_CHECK(launch_one(*sf, lm));
        LGF_HIP_CHECK(launch_one(cands[c], cands[c].mode));
        if (si) LGF_HIP_CHECK(launch_one(*si, lm));
        LGF_HIP_CHECK(hipEventRecord(b, st));
        LGF_HIP_CHECK(hipEventSynchronize(b));
        LGF_HIP_CHECK(hipEventElapsedTime(&t[rep], a, b));
      }
      std::sort(t, t + kTuneReps);
      if (verbose)
        std::fprintf(stderr, "[lgf tune] kind %d ty %d work %lld mode %d: %.1f us\n", cands[c].kind, cands[c].ty,
                     (long long)cands[c].work, cands[c].mode, 1e3f * t[kTuneReps / 2]);
      // an alternative replaces the planner's shape only when clearly faster (5%), so that
      // near ties do not flip from run to run
      if (c == 0 || t[kTuneReps / 2] < 0.95f * best) {
        best = t[kTuneReps / 2];
        best_i = c;
      }
    }
    choose(g.first, cands[best_i]);
    tune_store(key, cands[best_i].mode);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (din) {
    LGF_HIP_CHECK(hipStreamSynchronize(st));
    (void)hipFree(din);
  }
  sync_super_modes(p);
  return hipSuccess;
}

hipError_t plan_apply(Plan* p, int op, const double* u, double* out, hipStream_t st) {
  if (!p || p->dry || op < 0 || op > 2 || !u || !out) return hipErrorInvalidValue;
  return launch_fwd_op(p->nb, op, (const OpItem*)p->d_ops, p->nblocks, u, out, p->d_w3, st);
}

}  // namespace lgf
