// In-register radix-2 FFTs and the zero-padding-pruned transforms used by the block
// convolution (each line is held by one lane; LDS transposes happen in the callers).
#pragma once

#include "common.hpp"

namespace lgf {

template <int N> struct Log2;
template <> struct Log2<2> { static constexpr int v = 1; };
template <> struct Log2<4> { static constexpr int v = 2; };
template <> struct Log2<8> { static constexpr int v = 3; };
template <> struct Log2<16> { static constexpr int v = 4; };
template <> struct Log2<32> { static constexpr int v = 5; };
template <> struct Log2<64> { static constexpr int v = 6; };

constexpr int bitrev(int i, int bits) {
  int r = 0;
  for (int b = 0; b < bits; ++b) r |= ((i >> b) & 1) << (bits - 1 - b);
  return r;
}

template <int N> struct TwTable {
  static constexpr Turn<N> t{};
};

// In-place complex DFT of length N in natural order: X[k] = sum_n x[n] e^{SIGN 2 pi i n k / N}
// (SIGN = -1: forward, +1: inverse, unnormalised).  Fully unrolled: every twiddle is a literal.
template <int N, int SIGN, typename T>
__device__ __forceinline__ void fft_inreg(T (&re)[N], T (&im)[N]) {
  constexpr int B = Log2<N>::v;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const int j = bitrev(i, B);
    if (j > i) {
      T a = re[i]; re[i] = re[j]; re[j] = a;
      T b = im[i]; im[i] = im[j]; im[j] = b;
    }
  }
#pragma unroll
  for (int len = 2; len <= N; len <<= 1) {
    const int half = len >> 1;
    const int step = N / len;
#pragma unroll
    for (int i = 0; i < N; i += len) {
#pragma unroll
      for (int j = 0; j < half; ++j) {
        const int a = i + j, b = i + j + half;
        T br, bi;
        if (j == 0) {
          br = re[b]; bi = im[b];
        } else if (4 * j == len) {          // w = SIGN * i
          br = SIGN > 0 ? -im[b] : im[b];
          bi = SIGN > 0 ? re[b] : -re[b];
        } else {
          const T wr = T(TwTable<N>::t.c[j * step]);
          const T wi = T(SIGN * TwTable<N>::t.s[j * step]);
          br = re[b] * wr - im[b] * wi;
          bi = re[b] * wi + im[b] * wr;
        }
        re[b] = re[a] - br; im[b] = im[a] - bi;
        re[a] = re[a] + br; im[a] = im[a] + bi;
      }
    }
  }
}

// Forward DFT of length P = 2 NB of a line whose entries NB..P-1 are zero.
// Input x[0..NB) in (xr, xi); output X[0..P) in (Xr, Xi).
// X[2m] = DFT_NB(x)[m], X[2m+1] = DFT_NB(x[n] w^n)[m] with w = e^{-2 pi i / P}.
template <int NB, typename T>
__device__ __forceinline__ void fwd_padded(const T (&xr)[NB], const T (&xi)[NB], T (&Xr)[2 * NB],
                                           T (&Xi)[2 * NB]) {
  constexpr int P = 2 * NB;
  T er[NB], ei[NB], orr[NB], oi[NB];
#pragma unroll
  for (int n = 0; n < NB; ++n) {
    er[n] = xr[n]; ei[n] = xi[n];
    if (n == 0) {
      orr[n] = xr[n]; oi[n] = xi[n];
    } else {
      const T c = T(TwTable<P>::t.c[n]), s = T(-TwTable<P>::t.s[n]);
      orr[n] = xr[n] * c - xi[n] * s;
      oi[n] = xr[n] * s + xi[n] * c;
    }
  }
  fft_inreg<NB, -1>(er, ei);
  fft_inreg<NB, -1>(orr, oi);
#pragma unroll
  for (int m = 0; m < NB; ++m) {
    Xr[2 * m] = er[m]; Xi[2 * m] = ei[m];
    Xr[2 * m + 1] = orr[m]; Xi[2 * m + 1] = oi[m];
  }
}

// Inverse DFT of length P = 2 NB (unnormalised, e^{+2 pi i}) keeping outputs 0..NB-1 only.
// x[n] = IDFT_NB(X[2m])[n] + w^{-n} IDFT_NB(X[2m+1])[n].
template <int NB, typename T>
__device__ __forceinline__ void inv_cropped(const T (&Xr)[2 * NB], const T (&Xi)[2 * NB], T (&xr)[NB],
                                            T (&xi)[NB]) {
  constexpr int P = 2 * NB;
  T er[NB], ei[NB], orr[NB], oi[NB];
#pragma unroll
  for (int m = 0; m < NB; ++m) {
    er[m] = Xr[2 * m]; ei[m] = Xi[2 * m];
    orr[m] = Xr[2 * m + 1]; oi[m] = Xi[2 * m + 1];
  }
  fft_inreg<NB, +1>(er, ei);
  fft_inreg<NB, +1>(orr, oi);
#pragma unroll
  for (int n = 0; n < NB; ++n) {
    if (n == 0) {
      xr[n] = er[n] + orr[n];
      xi[n] = ei[n] + oi[n];
    } else {
      const T c = T(TwTable<P>::t.c[n]), s = T(TwTable<P>::t.s[n]);
      xr[n] = er[n] + (orr[n] * c - oi[n] * s);
      xi[n] = ei[n] + (orr[n] * s + oi[n] * c);
    }
  }
}

}  // namespace lgf
