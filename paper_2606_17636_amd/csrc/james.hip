// James vacuum boundary (Sec. 4): screening masses, the boundary
// convolution with the discrete Green's function tables, folding of the
// ghost potential into the second solve, and the one-time DGF construction.
//
// Ghost cells are the Dirichlet ghost cells of the problem grid in a fixed
// order (inner radial, outer radial, lower b, upper b).  Per mode m:
//   sigma^m_g = coup_out_g * Psi^m[adj_g] / (4 pi G)          (Eqs. charge_*)
//   Theta^m_t = sum_s Gt^m[t][s] sigma^m_s                     (Eqs. theta_*)
//   f2^m[cell] = f^m[cell] + sum_{g adjacent} coup_in_g Theta^m_g
// (the second solve has ghost potential -Theta; its known part moves to the
// right-hand side with the opposite sign).
#include "smg_internal.h"

namespace {

constexpr int kThreads = 256;

__global__ void k_screen(const int* __restrict__ adj, const double* __restrict__ coup, int n_g, int plane,
                         int M, const double2* __restrict__ psi, double inv4piG, double2* __restrict__ sigma) {
  const int m = blockIdx.y;
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < n_g; g += gridDim.x * blockDim.x) {
    const double2 v = psi[(size_t)m * plane + adj[g]];
    const double c = coup[g] * inv4piG;
    sigma[(size_t)m * n_g + g] = make_double2(c * v.x, c * v.y);
  }
}

// Theta = Gt sigma per mode: each wavefront takes kRowsPerWave output rows,
// lanes stride the rows (coalesced 512-byte reads of the FP64 table), sigma
// staged in LDS.  A round loads kColRounds values of every row of the wave
// (clamped indices, all issued before the first is used), so a row costs one
// memory latency per 64 kColRounds columns; each lane still sums its columns
// in ascending order.
constexpr int kRowsPerBlock = 16;
constexpr int kRowsPerWave = kRowsPerBlock / (kThreads / 64);
constexpr int kColRounds = 4;

__global__ void __launch_bounds__(kThreads) k_conv(const double* __restrict__ dgf, const double2* __restrict__ sigma,
                                                  double2* __restrict__ theta, int n_g) {
  extern __shared__ double2 sg[];
  const int m = blockIdx.y;
  const double2* s = sigma + (size_t)m * n_g;
  for (int t = threadIdx.x; t < n_g; t += blockDim.x) sg[t] = s[t];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double* G = dgf + (size_t)m * n_g * n_g;
  const int row0 = blockIdx.x * kRowsPerBlock + wave * kRowsPerWave;
  double ax[kRowsPerWave], ay[kRowsPerWave];
#pragma unroll
  for (int r = 0; r < kRowsPerWave; ++r) ax[r] = ay[r] = 0.0;
  for (int c0 = 0; c0 < n_g; c0 += 64 * kColRounds) {
    double w[kRowsPerWave][kColRounds];
#pragma unroll
    for (int r = 0; r < kRowsPerWave; ++r)
#pragma unroll
      for (int k = 0; k < kColRounds; ++k)
        w[r][k] = G[(size_t)min(row0 + r, n_g - 1) * n_g + min(c0 + lane + 64 * k, n_g - 1)];
#pragma unroll
    for (int k = 0; k < kColRounds; ++k) {
      const int c = c0 + lane + 64 * k;
      const double2 v = sg[min(c, n_g - 1)];
#pragma unroll
      for (int r = 0; r < kRowsPerWave; ++r) {
        const double wk = c < n_g ? w[r][k] : 0.0;
        ax[r] = fma(wk, v.x, ax[r]);
        ay[r] = fma(wk, v.y, ay[r]);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < kRowsPerWave; ++r) {
    double x = ax[r], y = ay[r];
    for (int o = 32; o > 0; o >>= 1) {
      x += __shfl_xor(x, o);
      y += __shfl_xor(y, o);
    }
    if (lane == 0 && row0 + r < n_g) theta[(size_t)m * n_g + row0 + r] = make_double2(x, y);
  }
}

__global__ void k_apply(const int* __restrict__ cells, const int* __restrict__ g0, const int* __restrict__ g1,
                        const double* __restrict__ c0, const double* __restrict__ c1, int n_cells, int plane,
                        int n_g, const double2* __restrict__ theta, const double2* __restrict__ f,
                        double2* __restrict__ f2) {
  const int m = blockIdx.y;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n_cells; t += gridDim.x * blockDim.x) {
    const size_t q = (size_t)m * plane + cells[t];
    double2 v = f[q];
    const double2 a = theta[(size_t)m * n_g + g0[t]];
    v.x = fma(c0[t], a.x, v.x);
    v.y = fma(c0[t], a.y, v.y);
    if (g1[t] >= 0) {
      const double2 b = theta[(size_t)m * n_g + g1[t]];
      v.x = fma(c1[t], b.x, v.x);
      v.y = fma(c1[t], b.y, v.y);
    }
    f2[q] = v;
  }
}

}  // namespace

namespace smgk {

hipError_t james_screen(const int* adj, const double* coup, int n_g, int plane, int M, const double2* psi,
                        double inv4piG, double2* sigma, hipStream_t st) {
  hipLaunchKernelGGL(k_screen, dim3((n_g + 255) / 256, M), dim3(256), 0, st, adj, coup, n_g, plane, M, psi,
                     inv4piG, sigma);
  return hipGetLastError();
}

hipError_t james_conv(const double* dgf, const double2* sigma, double2* theta, int n_g, int M, hipStream_t st) {
  hipLaunchKernelGGL(k_conv, dim3((n_g + kRowsPerBlock - 1) / kRowsPerBlock, M), dim3(kThreads),
                     sizeof(double2) * n_g, st, dgf, sigma, theta, n_g);
  return hipGetLastError();
}

hipError_t james_apply(const int* cells, const int* g0, const int* g1, const double* c0, const double* c1,
                          int n_cells, int plane, int n_g, int M, const double2* theta, const double2* f,
                          double2* f2, hipStream_t st) {
  hipLaunchKernelGGL(k_apply, dim3((n_cells + 255) / 256, M), dim3(256), 0, st, cells, g0, g1, c0, c1, n_cells,
                     plane, n_g, theta, f, f2);
  return hipGetLastError();
}

}  // namespace smgk
