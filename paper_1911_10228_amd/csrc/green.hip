// Lattice Green's function of the 7-point Laplacian on the GPU (FP64) and the kernel spectra of
// the block convolution.
//
// G(n) = -int_0^inf ive(n1,2t) ive(n2,2t) ive(n3,2t) dt  (Sec. 2, eq. GL_B, ive(k,x) = e^-x I_k(x))
// is evaluated by exp-sinh quadrature t = exp(pi/2 sinh u) on a uniform u grid (Takahasi & Mori
// 1974).  At every node the scaled Bessel functions of orders 0..100 come from
//   * the ascending series  I_k(x) = sum_j (x/2)^{2j+k} / (j! (j+k)!)      for x < 1/2,
//   * Miller's backward recurrence I_{k-1} = I_{k+1} + (2k/x) I_k normalised by
//     I_0 + 2 sum_k I_k = e^x                                                for 1/2 <= x < 4e4,
//   * the Hankel expansion (Abramowitz & Stegun 9.7.1)                      for x >= 4e4,
// and G of every sorted triple a >= b >= c with a^2+b^2+c^2 <= 100^2 is the compensated sum of the
// node products.  Outside the table the paper's policy applies: A_G^3 for 100 < |n| <= 600 and
// A_G^2 beyond (Sec. 2), with the degree-8 term of A_G^3 taken with a minus sign (the reading
// under which the expansion error decays like |n|^-7 as the paper states).
#include "kernels.hpp"

namespace lgf {

namespace {

constexpr int kQuadNodes = 1254;          // u in [-4.5, 5.3], step 1/128
constexpr double kQuadU0 = -4.5;
constexpr double kQuadH = 1.0 / 128.0;
constexpr double kHankelX = 4.0e4;

__global__ void bessel_nodes_kernel(double* __restrict__ tab /*[nodes][KMAX+1]*/,
                                    double* __restrict__ wts /*[nodes]*/) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= kQuadNodes) return;
  const double u = kQuadU0 + kQuadH * j;
  const double half_pi = 0.5 * kPi;
  const double t = exp(half_pi * sinh(u));
  wts[j] = kQuadH * half_pi * cosh(u) * t;
  const double x = 2.0 * t;
  double* row = tab + (size_t)j * (kTableKmax + 1);
  if (x < 0.5) {
    const double e = exp(-x);
    const double q = 0.25 * x * x;
    double lead = e;                        // e^-x (x/2)^k / k!
    for (int k = 0; k <= kTableKmax; ++k) {
      if (k > 0) lead *= 0.5 * x / k;
      double term = 1.0, sum = 1.0;
      for (int i = 1; i < 24; ++i) {
        term *= q / (double(i) * double(i + k));
        sum += term;
        if (term < 1e-18 * sum) break;
      }
      row[k] = lead * sum;
    }
  } else if (x < kHankelX) {
    const int N = kTableKmax + 40 + (int)(2.0 * sqrt(40.0 * x));
    double pk1 = 0.0, pk = 1e-280, norm = 0.0;
    for (int k = N; k >= 1; --k) {
      const double pm = pk1 + (2.0 * k / x) * pk;   // p_{k-1}
      if (k <= kTableKmax) row[k] = pk;
      norm += 2.0 * pk;
      pk1 = pk;
      pk = pm;
      if (fabs(pk) > 1e200) {
        pk *= 1e-200; pk1 *= 1e-200; norm *= 1e-200;
        for (int m = k; m <= kTableKmax; ++m) row[m] *= 1e-200;
      }
    }
    row[0] = pk;
    norm += pk;
    const double inv = 1.0 / norm;
    for (int k = 0; k <= kTableKmax; ++k) row[k] *= inv;
  } else {
    const double pref = 1.0 / sqrt(2.0 * kPi * x);
    for (int k = 0; k <= kTableKmax; ++k) {
      const double mu = 4.0 * k * k;
      double term = 1.0, sum = 1.0;
      for (int i = 1; i <= 20; ++i) {
        term *= -(mu - double((2 * i - 1) * (2 * i - 1))) / (8.0 * i * x);
        sum += term;
      }
      row[k] = pref * sum;
    }
  }
}

__global__ void green_table_kernel(const double* __restrict__ tab, const double* __restrict__ wts,
                                   const int16_t* __restrict__ triples, int ntri,
                                   double* __restrict__ cube) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ntri) return;
  const int a = triples[3 * i], b = triples[3 * i + 1], c = triples[3 * i + 2];
  double sum = 0.0, comp = 0.0;          // Kahan summation over the nodes
  for (int j = 0; j < kQuadNodes; ++j) {
    const double* row = tab + (size_t)j * (kTableKmax + 1);
    const double v = wts[j] * row[a] * row[b] * row[c];
    const double y = v - comp;
    const double s = sum + y;
    comp = (s - sum) - y;
    sum = s;
  }
  cube[((size_t)a * (kTableKmax + 1) + b) * (kTableKmax + 1) + c] = -sum;
}

__global__ void green_eval_kernel(const int32_t* __restrict__ n, int64_t m,
                                  const double* __restrict__ cube, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  out[i] = green(n[3 * i], n[3 * i + 1], n[3 * i + 2], cube);
}

// K[z][y][x] for one (s, d): G(s (d nb + r)) with r = idx (idx < nb), idx - P (idx > nb), 0 at nb
__global__ void kernel_fill_kernel(const int32_t* __restrict__ sd /*[nspec][4] = s,dx,dy,dz*/,
                                   int nb, const double* __restrict__ cube,
                                   double* __restrict__ out /*[nspec][P^3]*/) {
  const int P = 2 * nb;
  const int64_t P3 = (int64_t)P * P * P;
  const int spec = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P3) return;
  const int x = i % P, y = (i / P) % P, z = i / (P * P);
  const int s = sd[4 * spec], dx = sd[4 * spec + 1], dy = sd[4 * spec + 2], dz = sd[4 * spec + 3];
  double v = 0.0;
  if (x != nb && y != nb && z != nb) {
    const int rx = x < nb ? x : x - P, ry = y < nb ? y : y - P, rz = z < nb ? z : z - P;
    v = green(s * (dx * nb + rx), s * (dy * nb + ry), s * (dz * nb + rz), cube);
  }
  out[spec * P3 + i] = v;
}

// Full (unpruned) 3-D real-to-complex FFT of P^3 FP64 arrays, one lane per line, three passes
// through global memory (plan-time only).  Output layout [kz][ky][kx], kx in [0, P/2].
template <int P>
__global__ void full_fft_x(const double* __restrict__ in, c64* __restrict__ tmp, int nspec) {
  constexpr int H = P / 2 + 1;
  const int64_t line = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (line >= (int64_t)nspec * P * P) return;
  const double* src = in + line * P;
  double re[P], im[P];
#pragma unroll
  for (int i = 0; i < P; ++i) { re[i] = src[i]; im[i] = 0.0; }
  fft_inreg<P, -1>(re, im);
  c64* dst = tmp + line * H;            // [spec][z][y][kx]
#pragma unroll
  for (int k = 0; k < H; ++k) dst[k] = {re[k], im[k]};
}

template <int P>
__global__ void full_fft_y(c64* __restrict__ tmp, int nspec) {
  constexpr int H = P / 2 + 1;
  const int64_t line = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // (spec, z, kx)
  if (line >= (int64_t)nspec * P * H) return;
  const int kx = line % H;
  const int64_t sz = line / H;                                           // spec * P + z
  c64* base = tmp + sz * P * H + kx;
  double re[P], im[P];
#pragma unroll
  for (int y = 0; y < P; ++y) { re[y] = base[y * H].x; im[y] = base[y * H].y; }
  fft_inreg<P, -1>(re, im);
#pragma unroll
  for (int y = 0; y < P; ++y) base[y * H] = {re[y], im[y]};
}

template <int P>
__global__ void full_fft_z(const c64* __restrict__ tmp, c64* __restrict__ out64,
                           c32* __restrict__ out32, int nspec) {
  constexpr int H = P / 2 + 1;
  const int64_t line = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // (spec, ky, kx)
  if (line >= (int64_t)nspec * P * H) return;
  const int64_t spec = line / (P * H);
  const int rem = line % (P * H);                                        // ky * H + kx
  const c64* base = tmp + spec * P * P * H + rem;
  double re[P], im[P];
#pragma unroll
  for (int z = 0; z < P; ++z) { re[z] = base[(int64_t)z * P * H].x; im[z] = base[(int64_t)z * P * H].y; }
  fft_inreg<P, -1>(re, im);
  c64* o64 = out64 + spec * P * P * H + rem;
  c32* o32 = out32 ? out32 + spec * P * P * H + rem : nullptr;
#pragma unroll
  for (int z = 0; z < P; ++z) {
    o64[(int64_t)z * P * H] = {re[z], im[z]};
    if (o32) o32[(int64_t)z * P * H] = {float(re[z]), float(im[z])};
  }
}

// The same three passes for long lines: one workgroup of P lanes per line, lane k forms output k
// as a direct DFT from the line staged in LDS, with twiddles e^{-2 pi i m / P} from sincospi.
// PASS 0: real x-lines -> tmp[spec][z][y][kx]; PASS 1: y-lines of tmp in place; PASS 2: z-lines
// of tmp -> out[spec][kz][ky][kx].
template <int P, int PASS>
__global__ __launch_bounds__(P) void full_dft_lds(const double* __restrict__ in_real,
                                                  const c64* in_c, c64* out, c32* out32,
                                                  int nspec) {
  constexpr int H = P / 2 + 1;
  __shared__ double lr[P], li[P], wr[P], wi[P];
  const int64_t line = blockIdx.x;
  const int k = threadIdx.x;
  {
    double s, c;
    sincospi(-2.0 * k / P, &s, &c);
    wr[k] = c;
    wi[k] = s;
  }
  int64_t base, stride, obase, ostride;
  if (PASS == 0) {                     // line = (spec, z, y)
    base = line * P; stride = 1; obase = line * H; ostride = 1;
  } else if (PASS == 1) {              // line = (spec, z, kx)
    const int kx = line % H;
    base = (line / H) * P * H + kx; stride = H; obase = base; ostride = H;
  } else {                             // line = (spec, ky, kx)
    const int64_t spec = line / (P * H);
    base = spec * P * P * H + line % (P * H); stride = (int64_t)P * H; obase = base; ostride = stride;
  }
  if (PASS == 0) {
    lr[k] = in_real[base + k];
    li[k] = 0.0;
  } else {
    const c64 v = in_c[base + k * stride];
    lr[k] = v.x;
    li[k] = v.y;
  }
  __syncthreads();
  double sr = 0.0, si = 0.0;
  for (int j = 0; j < P; ++j) {
    const int m = (j * k) & (P - 1);
    sr += lr[j] * wr[m] - li[j] * wi[m];
    si += lr[j] * wi[m] + li[j] * wr[m];
  }
  if (PASS == 0 && k >= H) return;
  out[obase + k * ostride] = {sr, si};
  if (PASS == 2 && out32) out32[obase + k * ostride] = {float(sr), float(si)};
}

}  // namespace

int quad_nodes() { return kQuadNodes; }

hipError_t launch_green_table(double* d_cube, double* d_nodes, double* d_wts, const int16_t* d_tri,
                              int ntri, hipStream_t st) {
  bessel_nodes_kernel<<<(kQuadNodes + 63) / 64, 64, 0, st>>>(d_nodes, d_wts);
  LGF_HIP_CHECK(hipGetLastError());
  green_table_kernel<<<(ntri + 255) / 256, 256, 0, st>>>(d_nodes, d_wts, d_tri, ntri, d_cube);
  return hipGetLastError();
}

hipError_t launch_green_eval(const int32_t* d_n, int64_t m, const double* d_cube, double* d_out,
                             hipStream_t st) {
  if (m <= 0) return hipSuccess;
  green_eval_kernel<<<(unsigned)((m + 255) / 256), 256, 0, st>>>(d_n, m, d_cube, d_out);
  return hipGetLastError();
}

hipError_t launch_kernel_spectra(int nb, int nspec, const int32_t* d_sd, const double* d_cube,
                                 double* d_real, c64* d_tmp, c64* d_out64, c32* d_out32,
                                 hipStream_t st) {
  if (nspec <= 0) return hipSuccess;
  const int P = 2 * nb;
  const int64_t P3 = (int64_t)P * P * P;
  dim3 g((unsigned)((P3 + 255) / 256), (unsigned)nspec);
  kernel_fill_kernel<<<g, 256, 0, st>>>(d_sd, nb, d_cube, d_real);
  LGF_HIP_CHECK(hipGetLastError());
  const int H = P / 2 + 1;
  const int64_t lx = (int64_t)nspec * P * P, ly = (int64_t)nspec * P * H;
  if (P == 32) {
    full_fft_x<32><<<(unsigned)((lx + 63) / 64), 64, 0, st>>>(d_real, d_tmp, nspec);
    full_fft_y<32><<<(unsigned)((ly + 63) / 64), 64, 0, st>>>(d_tmp, nspec);
    full_fft_z<32><<<(unsigned)((ly + 63) / 64), 64, 0, st>>>(d_tmp, d_out64, d_out32, nspec);
  } else if (P == 16) {
    full_fft_x<16><<<(unsigned)((lx + 63) / 64), 64, 0, st>>>(d_real, d_tmp, nspec);
    full_fft_y<16><<<(unsigned)((ly + 63) / 64), 64, 0, st>>>(d_tmp, nspec);
    full_fft_z<16><<<(unsigned)((ly + 63) / 64), 64, 0, st>>>(d_tmp, d_out64, d_out32, nspec);
  } else if (P == 64) {
    // too long a line for one lane's registers: one workgroup per line, DFT through LDS
    full_dft_lds<64, 0><<<(unsigned)lx, 64, 0, st>>>(d_real, nullptr, d_tmp, nullptr, nspec);
    full_dft_lds<64, 1><<<(unsigned)ly, 64, 0, st>>>(nullptr, d_tmp, d_tmp, nullptr, nspec);
    full_dft_lds<64, 2><<<(unsigned)ly, 64, 0, st>>>(nullptr, d_tmp, d_out64, d_out32, nspec);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace lgf
