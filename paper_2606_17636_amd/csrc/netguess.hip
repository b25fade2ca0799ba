// The learned guess inside a solve: network inputs from the mode planes of
// modes 0..m_max (one image per real or imaginary part), the candidate
// u_prev + s_u * net(x), the choice per mode between it and the previous
// step's solution by their defect norms, training-sample recording, and the
// bookkeeping of the previous step's right-hand side.
#include "netguess.h"

namespace {

__device__ __forceinline__ double part_of(double2 v, int im) { return im ? v.y : v.x; }

// image k -> (mode, part): k = 0 -> (0, re); k = 2m - 1 -> (m, re); k = 2m -> (m, im)
__device__ __forceinline__ void image_mode(int k, int* m, int* im) {
  *m = (k + 1) / 2;
  *im = (k > 0 && (k & 1) == 0) ? 1 : 0;
}

// per image: RMS of f_t, of f_t - f_prev and of u_prev, and the output
// scale: sc = (s_f, s_d, s_u, s_o) with s_o = s_u s_d / s_f (the size the
// change of u takes when it follows the change of f); 1 where zero
__global__ void k_scales(const double2* __restrict__ f, const double2* __restrict__ fprev,
                         const double2* __restrict__ uprev, int plane, double* __restrict__ sc) {
  __shared__ double red[3][256];
  int m, im;
  image_mode(blockIdx.x, &m, &im);
  double a = 0.0, b = 0.0, c = 0.0;
  for (int t = threadIdx.x; t < plane; t += blockDim.x) {
    const double fv = part_of(f[(size_t)m * plane + t], im), uv = part_of(uprev[(size_t)m * plane + t], im);
    const double dv = fv - part_of(fprev[(size_t)m * plane + t], im);
    a += fv * fv;
    b += dv * dv;
    c += uv * uv;
  }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  red[2][threadIdx.x] = c;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
      for (int q = 0; q < 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double sf = sqrt(red[0][0] / plane), sd = sqrt(red[1][0] / plane), su = sqrt(red[2][0] / plane);
    sf = sf > 0.0 ? sf : 1.0;
    sd = sd > 0.0 ? sd : 1.0;
    su = su > 0.0 ? su : 1.0;
    sc[4 * blockIdx.x] = sf;
    sc[4 * blockIdx.x + 1] = sd;
    sc[4 * blockIdx.x + 2] = su;
    sc[4 * blockIdx.x + 3] = su * sd / sf;
  }
}

// x[k][i][j][0..7] = (f_t / s_f, (f_t - f_prev) / s_d, u_prev / s_u, m / 4,
//                     (i + 1/2) / n_a - 1/2, (j + 1/2) / n_b - 1/2,
//                     (u_prev - u_prev2) / s_o, 0)
// (channels 4, 5 tell the convolutions where on the grid they are;
// channel 6, the previous step's change of the solution, is zero when
// uprev2 is null: no solution two steps back)
__global__ void k_assemble(const double2* __restrict__ f, const double2* __restrict__ fprev,
                           const double2* __restrict__ uprev, const double2* __restrict__ uprev2,
                           const double* __restrict__ sc, int na, int nb, int n_img, float* __restrict__ x) {
  const int plane = na * nb;
  const size_t total = (size_t)n_img * plane;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
    const int k = (int)(t / plane), q = (int)(t - (size_t)k * plane);
    int m, im;
    image_mode(k, &m, &im);
    const double fv = part_of(f[(size_t)m * plane + q], im);
    const double fp = part_of(fprev[(size_t)m * plane + q], im);
    const double uv = part_of(uprev[(size_t)m * plane + q], im);
    const double sf = sc[4 * k], sd = sc[4 * k + 1], su = sc[4 * k + 2], so = sc[4 * k + 3];
    const double dv = uprev2 ? (uv - part_of(uprev2[(size_t)m * plane + q], im)) / so : 0.0;
    const int i = q / nb, j = q - i * nb;
    float4* xo = reinterpret_cast<float4*>(x) + 2 * t;
    xo[0] = make_float4((float)(fv / sf), (float)((fv - fp) / sd), (float)(uv / su), 0.25f * (float)m);
    xo[1] = make_float4((i + 0.5f) / na - 0.5f, (j + 0.5f) / nb - 0.5f, (float)dv, 0.f);
  }
}

// cand = u_prev + s_o * y, both parts of modes 0..m_max (m = 0 keeps its
// imaginary part)
__global__ void k_candidate(const double2* __restrict__ uprev, const float* __restrict__ y, const double* __restrict__ sc,
                            int plane, int m_max, double2* __restrict__ cand) {
  const size_t total = (size_t)(m_max + 1) * plane;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
    const int m = (int)(t / plane), q = (int)(t - (size_t)m * plane);
    double2 v = uprev[t];
    const int kr = m == 0 ? 0 : 2 * m - 1;
    v.x += sc[4 * kr + 3] * (double)y[(size_t)kr * plane + q];
    if (m > 0) v.y += sc[4 * (2 * m) + 3] * (double)y[(size_t)(2 * m) * plane + q];
    cand[t] = v;
  }
}

// per mode: keep the candidate where its defect norm is the smaller one
__global__ void k_select(const double* __restrict__ pc, const double* __restrict__ pu, int nblk,
                         const double2* __restrict__ cand, double2* __restrict__ u, int plane, int* __restrict__ used) {
  __shared__ int take;
  const int m = blockIdx.x;
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int k = 0; k < nblk; ++k) {
      a += pc[(size_t)m * nblk + k];
      b += pu[(size_t)m * nblk + k];
    }
    take = a < b ? 1 : 0;
    used[m] = take;
  }
  __syncthreads();
  if (!take) return;
  for (int t = threadIdx.x; t < plane; t += blockDim.x) u[(size_t)m * plane + t] = cand[(size_t)m * plane + t];
}

// training samples: (x, (u_t - u_prev) / s_o) per image at list position
// *count + k while below capacity
__global__ void k_record(const float* __restrict__ x, const double2* __restrict__ u, const double2* __restrict__ uprev,
                         const double* __restrict__ sc, int plane, int n_img, const int* __restrict__ count, int capacity,
                         float* __restrict__ samples) {
  const int base = *count;
  const size_t total = (size_t)n_img * plane;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
    const int k = (int)(t / plane), q = (int)(t - (size_t)k * plane);
    if (base + k >= capacity) continue;
    int m, im;
    image_mode(k, &m, &im);
    float* s = samples + (size_t)(base + k) * plane * 9;
    reinterpret_cast<float4*>(s)[2 * q] = reinterpret_cast<const float4*>(x)[2 * t];
    reinterpret_cast<float4*>(s)[2 * q + 1] = reinterpret_cast<const float4*>(x)[2 * t + 1];
    const double d = part_of(u[(size_t)m * plane + q], im) - part_of(uprev[(size_t)m * plane + q], im);
    s[(size_t)plane * 8 + q] = (float)(d / sc[4 * k + 3]);
  }
}

__global__ void k_advance(int* count, int n, int capacity) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *count = min(*count + n, capacity);
}

unsigned grid1(size_t n) {
  size_t g = (n + 255) / 256;
  return (unsigned)(g < 1 ? 1 : (g > 8192 ? 8192 : g));
}

}  // namespace

namespace smgg {

hipError_t scales(const double2* f, const double2* fprev, const double2* uprev, int plane, int n_img, double* sc,
                  hipStream_t st) {
  hipLaunchKernelGGL(k_scales, dim3(n_img), dim3(256), 0, st, f, fprev, uprev, plane, sc);
  return hipGetLastError();
}

hipError_t assemble(const double2* f, const double2* fprev, const double2* uprev, const double2* uprev2, const double* sc,
                    int na, int nb, int n_img, float* x, hipStream_t st) {
  hipLaunchKernelGGL(k_assemble, dim3(grid1((size_t)n_img * na * nb)), dim3(256), 0, st, f, fprev, uprev, uprev2, sc, na,
                     nb, n_img, x);
  return hipGetLastError();
}

hipError_t candidate(const double2* uprev, const float* y, const double* sc, int plane, int m_max, double2* cand,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_candidate, dim3(grid1((size_t)(m_max + 1) * plane)), dim3(256), 0, st, uprev, y, sc, plane, m_max,
                     cand);
  return hipGetLastError();
}

hipError_t select(const double* pc, const double* pu, int nblk, const double2* cand, double2* u, int plane, int m_max,
                  int* used, hipStream_t st) {
  hipLaunchKernelGGL(k_select, dim3(m_max + 1), dim3(256), 0, st, pc, pu, nblk, cand, u, plane, used);
  return hipGetLastError();
}

hipError_t record(const float* x, const double2* u, const double2* uprev, const double* sc, int plane, int n_img,
                  int* count, int capacity, float* samples, hipStream_t st) {
  hipLaunchKernelGGL(k_record, dim3(grid1((size_t)n_img * plane)), dim3(256), 0, st, x, u, uprev, sc, plane, n_img, count,
                     capacity, samples);
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, st, count, n_img, capacity);
  return hipGetLastError();
}

}  // namespace smgg
