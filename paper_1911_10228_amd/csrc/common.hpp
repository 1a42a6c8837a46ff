// Shared device/host helpers of the LGF library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#define LGF_HIP_CHECK(expr)                                  \
  do {                                                       \
    hipError_t e_ = (expr);                                  \
    if (e_ != hipSuccess) return e_;                         \
  } while (0)

namespace lgf {

template <typename T> struct cpx { T x, y; };
using c32 = cpx<float>;
using c64 = cpx<double>;

template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// acc += a * b (complex)
template <typename T>
__device__ __forceinline__ void cmac(cpx<T>& acc, cpx<T> a, cpx<T> b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}

// Global-memory views of generic pointers.  Accesses through them compile to global_* rather
// than flat_* instructions; a flat access also counts against the LDS/scalar wait counter, so in
// a kernel that mixes memory and LDS traffic every wait for an LDS result would also wait for all
// memory accesses still in flight.
template <typename T> using gview = __attribute__((address_space(1))) T*;
template <typename T> __device__ __forceinline__ gview<T> gl(T* p) { return (gview<T>)p; }
// complex element i of a global array (as two scalars: class assignment has no global form)
template <typename T> __device__ __forceinline__ cpx<T> gld(const cpx<T>* p, int64_t i) {
  const gview<const T> q = gl((const T*)p);
  return {q[2 * i], q[2 * i + 1]};
}
template <typename T> __device__ __forceinline__ void gst(cpx<T>* p, int64_t i, cpx<T> v) {
  const gview<T> q = gl((T*)p);
  q[2 * i] = v.x;
  q[2 * i + 1] = v.y;
}

// ---------------------------------------------------------------------------------------------
// Compile-time twiddle factors cos/sin(2 pi m / N), from Taylor series on the first octant and
// the exact symmetries of the circle (no math-library constants involved).
constexpr double kPi = 3.141592653589793238462643383279502884;

constexpr double taylor_sin(double x) {
  double x2 = x * x, term = x, sum = x;
  for (int i = 1; i < 14; ++i) {
    term *= -x2 / double((2 * i) * (2 * i + 1));
    sum += term;
  }
  return sum;
}
constexpr double taylor_cos(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int i = 1; i < 14; ++i) {
    term *= -x2 / double((2 * i - 1) * (2 * i));
    sum += term;
  }
  return sum;
}
// cos(2 pi m / N) and sin(2 pi m / N) for 0 <= m < N, N divisible by 8
constexpr double turn_cos(long m, long N);
constexpr double turn_sin(long m, long N) {
  m = ((m % N) + N) % N;
  if (2 * m > N) return -turn_sin(N - m, N);               // (pi, 2pi): sin(2pi - t) = -sin t
  if (4 * m > N) return turn_sin(N / 2 - m, N);            // (pi/2, pi]: sin(pi - t) = sin t
  if (8 * m > N) return turn_cos(N / 4 - m, N);            // (pi/4, pi/2]: sin t = cos(pi/2 - t)
  return taylor_sin(2.0 * kPi * double(m) / double(N));
}
constexpr double turn_cos(long m, long N) {
  m = ((m % N) + N) % N;
  if (2 * m > N) return turn_cos(N - m, N);
  if (4 * m > N) return -turn_cos(N / 2 - m, N);
  if (8 * m > N) return turn_sin(N / 4 - m, N);
  return taylor_cos(2.0 * kPi * double(m) / double(N));
}

template <int N> struct Turn {
  double c[N];
  double s[N];
  constexpr Turn() : c{}, s{} {
    for (int m = 0; m < N; ++m) {
      c[m] = turn_cos(m, N);
      s[m] = turn_sin(m, N);
    }
  }
};

// ---------------------------------------------------------------------------------------------
// Work sets: one kernel launch can process items of several plans (batched solves).  Each set
// names an item array in device memory and the number of workgroups its items need; a
// workgroup finds its set by scanning the prefix sums (few sets per launch).
constexpr int kMaxSets = 48;

struct WorkSet {
  const void* items;   // device array of per-kernel item structs
  int64_t wg_begin;    // first workgroup of this set
  int32_t count;       // number of items
  int32_t aux;         // flags: kAuxAccumulate
  const double* in;    // the solve pass's input field (items address it by offset)
  double* out;         // the solve pass's output field
  const double* w;     // the plan's 1-D weight table of this kernel
};

// WorkSet::aux: the combine adds into the output field instead of writing it (the pass is a
// defect-correction re-solve whose result updates u)
constexpr int32_t kAuxAccumulate = 1;

struct SetTable {
  int32_t n;
  int32_t pad;
  WorkSet s[kMaxSets];
};

__device__ __forceinline__ int find_set(const SetTable& t, int64_t wg) {
  int lo = 0;
  for (int i = 1; i < t.n; ++i)
    if (t.s[i].wg_begin <= wg) lo = i;
  return lo;
}

}  // namespace lgf
