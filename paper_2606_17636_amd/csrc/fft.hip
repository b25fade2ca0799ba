// Azimuthal real FFT (Sec. 2.2 and step 2 / step 7 of Sec. 5.1).
//
// Forward: modes[m][line] = scale * sum_k rho[line][k] e^{-2 pi i m k / N},
// m = 0..N/2, line = i*n_b + j (so mode m's output is the contiguous plane
// [n_a][n_b]), optionally written to a second array as well.  Inverse:
// out[line][k] = sum_{m=0}^{N-1} X_m e^{+2 pi i m k/N} with Hermitian
// completion.
//
// A real line of length N is packed as n = N/2 complex values
// z_k = x_{2k} + i x_{2k+1}; an n-point complex Stockham FFT (radices 4, 2,
// 3) runs in LDS, and the two interleaved half-length spectra are separated
// with the post-twiddles e^{-2 pi i m / N}.  A block handles lpb consecutive
// lines (a launch parameter), which are contiguous in the input and give
// contiguous segments of every output plane.  Twiddles come from a table built on the host in FP64.
#include <algorithm>

#include "smg_internal.h"

namespace {

constexpr int kThreads = 256;
constexpr int kPoints = 1024;  // complex points staged per block (ping-pong)
// Values a thread moves per round of the staging and output loops: every
// global load of a round is issued, unconditionally from an index clamped
// into the array, before the first of them is used, so a round costs one
// memory latency (a loop with a runtime trip count would wait for each load
// in turn).
constexpr int kItems = kPoints / kThreads;

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
// multiply by -i
__device__ __forceinline__ double2 cmi(double2 a) { return make_double2(a.y, -a.x); }

// One Stockham pass of radix R over LPB lines of n points: src -> dst.
template <int R>
__device__ void stockham_pass(const double2* __restrict__ src, double2* __restrict__ dst, int n, int lines,
                              int Ns, const double2* __restrict__ tw) {
  const int nb = n / R;
  const int total = lines * nb;
  for (int b = threadIdx.x; b < total; b += blockDim.x) {
    const int line = b / nb, j = b - line * nb;
    const double2* s = src + line * n;
    double2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = s[j + r * nb];
    const int k = j % Ns;
    if (Ns > 1) {
      const int step = n / (Ns * R);
#pragma unroll
      for (int r = 1; r < R; ++r) v[r] = cmul(v[r], tw[(r * k * step) % n]);
    }
    if (R == 2) {
      double2 a = v[0], c = v[1];
      v[0] = cadd(a, c);
      v[1] = csub(a, c);
    } else if (R == 4) {
      double2 a0 = v[0], a1 = v[1], a2 = v[2], a3 = v[3];
      double2 s02 = cadd(a0, a2), d02 = csub(a0, a2);
      double2 s13 = cadd(a1, a3), d13 = cmi(csub(a1, a3));
      v[0] = cadd(s02, s13);
      v[2] = csub(s02, s13);
      v[1] = cadd(d02, d13);
      v[3] = csub(d02, d13);
    } else {  // R == 3
      const double h = 0.86602540378443864676372317075294;  // sqrt(3)/2
      double2 a0 = v[0], a1 = v[1], a2 = v[2];
      double2 t1 = cadd(a1, a2);
      double2 t2 = make_double2(a0.x - 0.5 * t1.x, a0.y - 0.5 * t1.y);
      double2 d = csub(a1, a2);
      double2 t3 = make_double2(h * d.y, -h * d.x);  // -i sqrt(3)/2 (a1 - a2)
      v[0] = cadd(a0, t1);
      v[1] = cadd(t2, t3);
      v[2] = csub(t2, t3);
    }
    double2* d = dst + line * n;
    const int idxD = (j / Ns) * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) d[idxD + r * Ns] = v[r];
  }
}

// Full n-point forward complex FFT of `lines` lines in LDS; returns the
// buffer holding the result.
__device__ double2* fft_lds(double2* a, double2* b, int n, int lines, const double2* tw) {
  int Ns = 1;
  int rem = n;
  while (rem > 1) {
    if (rem % 4 == 0) {
      stockham_pass<4>(a, b, n, lines, Ns, tw);
      Ns *= 4; rem /= 4;
    } else if (rem % 2 == 0) {
      stockham_pass<2>(a, b, n, lines, Ns, tw);
      Ns *= 2; rem /= 2;
    } else {
      stockham_pass<3>(a, b, n, lines, Ns, tw);
      Ns *= 3; rem /= 3;
    }
    __syncthreads();
    double2* t = a; a = b; b = t;
  }
  return a;
}

__global__ void __launch_bounds__(kThreads) k_fft_r2c(const double* __restrict__ rho, double2* __restrict__ modes,
                                                     double2* __restrict__ modes2, int n_lines, int N, double scale,
                                                     const double2* __restrict__ tw, int lpb) {
  extern __shared__ double2 sh[];
  const int n = N / 2;
  double2* a = sh;
  double2* b = sh + lpb * n;
  const int line0 = blockIdx.x * lpb;
  const int lines = min(lpb, n_lines - line0);
  const double2* src = reinterpret_cast<const double2*>(rho + (size_t)line0 * N);
  for (int t0 = 0; t0 < lines * n; t0 += kItems * kThreads) {
    // clamped stores too (a thread past the end rewrites the last value with
    // itself), so that no load is sunk into a conditional store's branch
    double2 v[kItems];
#pragma unroll
    for (int r = 0; r < kItems; ++r) v[r] = src[min(t0 + (int)threadIdx.x + r * kThreads, lines * n - 1)];
#pragma unroll
    for (int r = 0; r < kItems; ++r) a[min(t0 + (int)threadIdx.x + r * kThreads, lines * n - 1)] = v[r];
  }
  __syncthreads();
  double2* z = fft_lds(a, b, n, lines, tw);
  // separate the even/odd half spectra: X_m = E_m + e^{-2 pi i m/N} O_m
  const double2* post = tw + n;
  const int total = lines * (n + 1);
  constexpr int kOut = kItems + 1;  // lines * (n + 1) <= kPoints + lines
  for (int t0 = 0; t0 < total; t0 += kOut * kThreads) {
    double2 pw[kOut];
#pragma unroll
    for (int r = 0; r < kOut; ++r) pw[r] = post[min(t0 + (int)threadIdx.x + r * kThreads, total - 1) / lines];
    __builtin_amdgcn_sched_barrier(0);  // the twiddle loads stay ahead of the arithmetic
#pragma unroll
    for (int r = 0; r < kOut; ++r) {
      const int t = t0 + threadIdx.x + r * kThreads;
      if (t >= total) continue;
      const int m = t / lines, line = t - m * lines;
      const double2* Z = z + line * n;
      double2 zm = Z[m % n];
      double2 zc = cconj(Z[(n - m) % n]);
      double2 E = make_double2(0.5 * (zm.x + zc.x), 0.5 * (zm.y + zc.y));
      double2 dd = csub(zm, zc);
      double2 O = make_double2(0.5 * dd.y, -0.5 * dd.x);  // -i/2 (Z_m - conj Z_{n-m})
      double2 X = cadd(E, cmul(pw[r], O));
      const double2 v = make_double2(scale * X.x, scale * X.y);
      modes[(size_t)m * n_lines + line0 + line] = v;
      if (modes2) modes2[(size_t)m * n_lines + line0 + line] = v;
    }
  }
}

__global__ void __launch_bounds__(kThreads) k_fft_c2r(const double2* __restrict__ modes, double* __restrict__ out,
                                                     int n_lines, int N, const double2* __restrict__ tw, int lpb) {
  extern __shared__ double2 sh[];
  const int n = N / 2;
  double2* a = sh;
  double2* b = sh + lpb * n;
  const int line0 = blockIdx.x * lpb;
  const int lines = min(lpb, n_lines - line0);
  const double2* post = tw + n;
  // Z_m = (X_m + conj X_{n-m}) + i w^m (X_m - conj X_{n-m}), w = e^{+2 pi i/N};
  // stored conjugated so that a forward FFT gives conj of the inverse sum.
  const int total = lines * n;
  for (int t0 = 0; t0 < total; t0 += kItems * kThreads) {
    double2 xm[kItems], xr[kItems], pw[kItems];
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      const int t = min(t0 + (int)threadIdx.x + r * kThreads, total - 1);
      const int m = t / lines, line = t - m * lines;
      xm[r] = modes[(size_t)m * n_lines + line0 + line];
      xr[r] = modes[(size_t)(n - m) * n_lines + line0 + line];
      pw[r] = post[m];
    }
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      const int t = t0 + threadIdx.x + r * kThreads;
      if (t >= total) continue;
      const int m = t / lines, line = t - m * lines;
      if (m == 0) { xm[r].y = 0.0; xr[r].y = 0.0; }  // m = 0 and m = N/2 are real
      double2 xc = cconj(xr[r]);
      double2 S = cadd(xm[r], xc);
      double2 D = csub(xm[r], xc);
      double2 wm = cconj(pw[r]);                 // e^{+2 pi i m/N}
      double2 iwD = cmul(make_double2(-wm.y, wm.x), D);  // i w^m D
      double2 Z = cadd(S, iwD);
      a[line * n + m] = cconj(Z);
    }
  }
  __syncthreads();
  double2* z = fft_lds(a, b, n, lines, tw);
  double2* dst = reinterpret_cast<double2*>(out + (size_t)line0 * N);
  for (int t = threadIdx.x; t < lines * n; t += blockDim.x) dst[t] = cconj(z[t]);
}

}  // namespace

namespace smgk {

// Lines per block: as many as the LDS budget (kPoints complex points, ping
// and pong) holds, but no more than gives kMinBlocks blocks, so that small
// transforms still spread over the device.
constexpr int kMinBlocks = 1024;
static int fft_lines_per_block(int n_lines, int n) {
  const int cap = kPoints / n;
  const int want = std::max(1, n_lines / kMinBlocks);
  return std::max(1, std::min(cap, want));
}

hipError_t fft_r2c(const double* rho, double2* modes, int n_lines, int n_phi, double scale,
                   const double2* tw, hipStream_t st, double2* modes2) {
  const int n = n_phi / 2, lpb = fft_lines_per_block(n_lines, n);
  const int blocks = (n_lines + lpb - 1) / lpb;
  hipLaunchKernelGGL(k_fft_r2c, dim3(blocks), dim3(kThreads), 2 * lpb * n * sizeof(double2), st, rho, modes, modes2,
                     n_lines, n_phi, scale, tw, lpb);
  return hipGetLastError();
}

hipError_t fft_c2r(const double2* modes, double* out, int n_lines, int n_phi, const double2* tw,
                   hipStream_t st) {
  const int n = n_phi / 2, lpb = fft_lines_per_block(n_lines, n);
  const int blocks = (n_lines + lpb - 1) / lpb;
  hipLaunchKernelGGL(k_fft_c2r, dim3(blocks), dim3(kThreads), 2 * lpb * n * sizeof(double2), st, modes, out,
                     n_lines, n_phi, tw, lpb);
  return hipGetLastError();
}

}  // namespace smgk
