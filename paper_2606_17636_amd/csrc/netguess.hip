// The learned guess inside a solve: network inputs from the mode planes of
// modes 0..m_max (one image per real or imaginary part), the candidate
// (linear extrapolation of the last two solutions + s_o * net(x)), the choice per mode between it and the
// extrapolation alone (the previous step's solution before two exist) by their defect norms, training-sample
// recording, and the
// bookkeeping of the previous step's right-hand side.  Also the extrapolated
// warm start of the modes the network does not handle.
#include "netguess.h"

#include <algorithm>

namespace {

// relative size of the last change below which a plane counts as static
// (a change that small leaves the previous solution a better start than
// any guess needs to be)
constexpr double kStatic = 1e-4;

__device__ __forceinline__ double part_of(double2 v, int im) { return im ? v.y : v.x; }

// image k -> (mode, part): k = 0 -> (0, re); k = 2m - 1 -> (m, re); k = 2m -> (m, im)
__device__ __forceinline__ void image_mode(int k, int* m, int* im) {
  *m = (k + 1) / 2;
  *im = (k > 0 && (k & 1) == 0) ? 1 : 0;
}

// Per image: RMS of f_t, of f_t - f_prev and of u_prev, and the output
// scale: sc = (s_f, s_d, s_u, s_o) with s_o the RMS of u_prev - u_prev2
// (the size of the last change of u) when u_prev2 is given, else
// s_u s_d / s_f (the size the change of u takes when it follows the change
// of f); 1 where zero.  Two passes: kScaleBlocks blocks per image write
// partial sums of squares (part[image][block][4]), one block per image then
// adds them in block order.
constexpr int kScaleBlocks = 32;

__global__ void k_scales_partial(const double2* __restrict__ f, const double2* __restrict__ fprev,
                                 const double2* __restrict__ uprev, const double2* __restrict__ uprev2, int plane,
                                 double* __restrict__ part) {
  __shared__ double red[4][256];
  int m, im;
  image_mode(blockIdx.y, &m, &im);
  double a = 0.0, b = 0.0, c = 0.0, e = 0.0;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < plane; t += gridDim.x * blockDim.x) {
    const double fv = part_of(f[(size_t)m * plane + t], im), uv = part_of(uprev[(size_t)m * plane + t], im);
    const double dv = fv - part_of(fprev[(size_t)m * plane + t], im);
    a += fv * fv;
    b += dv * dv;
    c += uv * uv;
    if (uprev2) {
      const double ev = uv - part_of(uprev2[(size_t)m * plane + t], im);
      e += ev * ev;
    }
  }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  red[2][threadIdx.x] = c;
  red[3][threadIdx.x] = e;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
      for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x < 4) part[((size_t)blockIdx.y * gridDim.x + blockIdx.x) * 4 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void k_scales_final(const double* __restrict__ part, int nblk, int plane, int have2, double* __restrict__ sc) {
  if (threadIdx.x != 0) return;
  double r[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k = 0; k < nblk; ++k)
    for (int q = 0; q < 4; ++q) r[q] += part[((size_t)blockIdx.x * nblk + k) * 4 + q];
  double sf = sqrt(r[0] / plane), sd = sqrt(r[1] / plane), su = sqrt(r[2] / plane);
  const double se = sqrt(r[3] / plane);
  sf = sf > 0.0 ? sf : 1.0;
  sd = sd > 0.0 ? sd : 1.0;
  su = su > 0.0 ? su : 1.0;
  sc[4 * blockIdx.x] = sf;
  sc[4 * blockIdx.x + 1] = sd;
  sc[4 * blockIdx.x + 2] = su;
  // a plane whose last change is at the level of the solve's own error
  // (below 1e-6 of the plane) is static: s_o = 0 marks it (no
  // extrapolation, no correction, no change channels, zero target)
  sc[4 * blockIdx.x + 3] = have2 ? (se > kStatic * su ? se : 0.0) : su * sd / sf;
}

// x[k][i][j][0..7] = (f_t / s_f, (f_t - f_prev) / s_d, u_prev / s_u, m / 4,
//                     (i + 1/2) / n_a - 1/2, (j + 1/2) / n_b - 1/2,
//                     this part of (u_prev - u_prev2) / s_o,
//                     this part of -i (u_prev - u_prev2) / s_o)
// (channels 4, 5 tell the convolutions where on the grid they are;
// channels 6, 7, the previous step's change of the solution, are zero when
// uprev2 is null or the plane is static)
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
    // the last change of u and of the partner part, as the corresponding
    // part of -i (u_prev - u_prev2): a rotation of the mode by a small
    // angle changes each part by that angle times it (zero for m = 0)
    double dv = 0.0, dr = 0.0;
    if (uprev2 && so > 0.0) {
      const double2 d2 = uprev[(size_t)m * plane + q], w2 = uprev2[(size_t)m * plane + q];
      const double re = d2.x - w2.x, imv = d2.y - w2.y;
      dv = (im ? imv : re) / so;
      dr = m > 0 ? (im ? -re : imv) / so : 0.0;
    }
    const int i = q / nb, j = q - i * nb;
    float4* xo = reinterpret_cast<float4*>(x) + 2 * t;
    xo[0] = make_float4((float)(fv / sf), (float)((fv - fp) / sd), (float)(uv / su), 0.25f * (float)m);
    xo[1] = make_float4((i + 0.5f) / na - 0.5f, (j + 0.5f) / nb - 0.5f, (float)dv, (float)dr);
  }
}

// The baseline of value t (mode m = t / plane): u_prev + (u_prev -
// u_prev2), the linear extrapolation of the last two solutions (u_prev alone
// when there is no u_prev2, or where the part is static: s_o = 0; the
// imaginary part of m = 0 has no image and follows the real part's kind)
__device__ __forceinline__ double2 guess_base(const double2* __restrict__ uprev, const double2* __restrict__ uprev2,
                                              const double* __restrict__ sc, int m, size_t t, double& sr, double& si) {
  double2 v = uprev[t];
  const int kr = m == 0 ? 0 : 2 * m - 1;
  sr = sc[4 * kr + 3];
  si = m > 0 ? sc[4 * (2 * m) + 3] : sr;
  if (uprev2) {
    const double2 w = uprev2[t];
    if (sr > 0.0) v.x += v.x - w.x;
    if (si > 0.0) v.y += v.y - w.y;
  }
  return v;
}

// cand = base + s_o * y (the network's correction), both parts of modes
// 0..m_max (m = 0 has no imaginary image: its imaginary part is only
// extrapolated); base = the baseline alone, the judge's other start
__global__ void k_candidate(const double2* __restrict__ uprev, const double2* __restrict__ uprev2,
                            const float* __restrict__ y, const double* __restrict__ sc, int plane, int m_max,
                            double2* __restrict__ cand, double2* __restrict__ base, double2* __restrict__ cand2) {
  const size_t total = (size_t)(m_max + 1) * plane;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
    const int m = (int)(t / plane), q = (int)(t - (size_t)m * plane);
    double sr, si;
    double2 v = guess_base(uprev, uprev2, sc, m, t, sr, si);
    base[t] = v;
    const int kr = m == 0 ? 0 : 2 * m - 1;
    v.x += sr * (double)y[(size_t)kr * plane + q];
    if (m > 0) v.y += si * (double)y[(size_t)(2 * m) * plane + q];
    cand[t] = v;
    if (cand2) cand2[t] = v;
  }
}

// per mode: the candidate where its defect norm is the smaller one, else
// the baseline (recomputed, with the arithmetic of k_candidate), or, with no
// uprev, u as it is (the other start was u itself).  Grid (blocks per plane,
// m_max + 1): every block sums its mode's partial norms (nblk each) and
// writes its slice of the plane; block 0 of the mode records the choice.
__global__ void k_select(const double* __restrict__ pc, const double* __restrict__ pu, int nblk,
                         const double2* __restrict__ cand, const double2* __restrict__ uprev,
                         const double2* __restrict__ uprev2, const double* __restrict__ sc, double2* __restrict__ u,
                         int plane, int* __restrict__ used) {
  __shared__ int take;
  const int m = blockIdx.y;
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int k = 0; k < nblk; ++k) {
      a += pc[(size_t)m * nblk + k];
      b += pu[(size_t)m * nblk + k];
    }
    take = a < b ? 1 : 0;
    if (blockIdx.x == 0) used[m] = take;
  }
  __syncthreads();
  if (!take && !uprev) return;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < plane; t += gridDim.x * blockDim.x) {
    const size_t k = (size_t)m * plane + t;
    double sr, si;
    u[k] = take ? cand[k] : guess_base(uprev, uprev2, sc, m, k, sr, si);
  }
}

// training samples: (x, (u_t - u_prev - (u_prev - u_prev2)) / s_o) per
// image (the correction the candidate needs; without u_prev2 the change
// u_t - u_prev) at list position *count + k while below capacity
__global__ void k_record(const float* __restrict__ x, const double2* __restrict__ u, const double2* __restrict__ uprev,
                         const double2* __restrict__ uprev2, const double* __restrict__ sc, int plane, int n_img,
                         const int* __restrict__ count, int capacity, float* __restrict__ samples) {
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
    const double up = part_of(uprev[(size_t)m * plane + q], im), so = sc[4 * k + 3];
    double d = part_of(u[(size_t)m * plane + q], im) - up;
    if (uprev2) d -= up - part_of(uprev2[(size_t)m * plane + q], im);
    s[(size_t)plane * 8 + q] = so > 0.0 ? (float)(d / so) : 0.f;
  }
}

__global__ void k_advance(int* count, int n, int capacity) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *count = min(*count + n, capacity);
}

// Warm start from the last k solutions, u (the latest) and the kept ones
// h[0], h[1], h[2] (older in turn; `kept` of them): from value lo on, u <-
// the value at the next step of the polynomial through them (k = 2:
// 2 u - h0; k = 3: 3 u - 3 h0 + h1; k = 4: 4 u - 6 h0 + 4 h1 - h2; k = 1: u
// unchanged); u's old value goes into h[kept - 1], the oldest position,
// whose slot the caller then makes the newest (a ring: nothing else moves).
struct History {
  double2* h[3];
};

// One value per thread (the pass is a stream over HBM: up to four plane sets read,
// two written); the kept solutions are read and written with non-temporal
// hints, since the next use of each is a step away, while u stays cached
// for the defect pass that follows.
typedef double cd2 __attribute__((ext_vector_type(2)));
template <int K>
__global__ void __launch_bounds__(256) k_extrapolate(double2* __restrict__ u, History hs, int kept, size_t n,
                                                     size_t lo) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const double2 x = u[t];
  cd2 q[3] = {};
#pragma unroll
  for (int j = 0; j < K - 1; ++j) q[j] = __builtin_nontemporal_load(reinterpret_cast<const cd2*>(hs.h[j]) + t);
  if (K >= 2 && t >= lo) {
    double2 v;
    if (K == 2) {
      v = make_double2(2.0 * x.x - q[0].x, 2.0 * x.y - q[0].y);
    } else if (K == 3) {
      v = make_double2(3.0 * (x.x - q[0].x) + q[1].x, 3.0 * (x.y - q[0].y) + q[1].y);
    } else {
      v = make_double2(4.0 * (x.x + q[1].x) - 6.0 * q[0].x - q[2].x, 4.0 * (x.y + q[1].y) - 6.0 * q[0].y - q[2].y);
    }
    u[t] = v;
  }
  cd2 keep;
  keep.x = x.x;
  keep.y = x.y;
  __builtin_nontemporal_store(keep, reinterpret_cast<cd2*>(hs.h[kept - 1]) + t);
}

unsigned grid1(size_t n) {
  size_t g = (n + 255) / 256;
  return (unsigned)(g < 1 ? 1 : (g > 8192 ? 8192 : g));
}

}  // namespace

namespace smgg {

size_t scales_partial_doubles(int n_img) { return (size_t)n_img * kScaleBlocks * 4; }

hipError_t scales(const double2* f, const double2* fprev, const double2* uprev, const double2* uprev2, int plane, int n_img,
                  double* part, double* sc, hipStream_t st) {
  hipLaunchKernelGGL(k_scales_partial, dim3(kScaleBlocks, n_img), dim3(256), 0, st, f, fprev, uprev, uprev2, plane, part);
  hipLaunchKernelGGL(k_scales_final, dim3(n_img), dim3(64), 0, st, part, kScaleBlocks, plane, uprev2 ? 1 : 0, sc);
  return hipGetLastError();
}

hipError_t assemble(const double2* f, const double2* fprev, const double2* uprev, const double2* uprev2, const double* sc,
                    int na, int nb, int n_img, float* x, hipStream_t st) {
  hipLaunchKernelGGL(k_assemble, dim3(grid1((size_t)n_img * na * nb)), dim3(256), 0, st, f, fprev, uprev, uprev2, sc, na,
                     nb, n_img, x);
  return hipGetLastError();
}

hipError_t candidate(const double2* uprev, const double2* uprev2, const float* y, const double* sc, int plane, int m_max,
                     double2* cand, double2* base, hipStream_t st, double2* cand2) {
  hipLaunchKernelGGL(k_candidate, dim3(grid1((size_t)(m_max + 1) * plane)), dim3(256), 0, st, uprev, uprev2, y, sc, plane,
                     m_max, cand, base, cand2);
  return hipGetLastError();
}

hipError_t select(const double* pc, const double* pu, int nblk, const double2* cand, const double2* uprev,
                  const double2* uprev2, const double* sc, double2* u, int plane, int m_max, int* used, hipStream_t st) {
  const int per = std::max(1, std::min(64, (plane + 1023) / 1024));
  hipLaunchKernelGGL(k_select, dim3(per, m_max + 1), dim3(256), 0, st, pc, pu, nblk, cand, uprev, uprev2, sc, u, plane,
                     used);
  return hipGetLastError();
}

hipError_t record(const float* x, const double2* u, const double2* uprev, const double2* uprev2, const double* sc,
                  int plane, int n_img, int* count, int capacity, float* samples, hipStream_t st) {
  hipLaunchKernelGGL(k_record, dim3(grid1((size_t)n_img * plane)), dim3(256), 0, st, x, u, uprev, uprev2, sc, plane, n_img,
                     count, capacity, samples);
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, st, count, n_img, capacity);
  return hipGetLastError();
}

hipError_t extrapolate(double2* u, double2* const* hist, int kept, size_t n, size_t lo, int k, hipStream_t st) {
  if (n == 0) return hipSuccess;
  if (kept < 1 || kept > 3 || k < 1 || k > kept + 1 || (n + 255) / 256 > 0x7fffffffu) return hipErrorInvalidValue;
  History hs{{nullptr, nullptr, nullptr}};
  for (int j = 0; j < kept; ++j) hs.h[j] = hist[j];
  const dim3 grid((unsigned)((n + 255) / 256));
  switch (k) {
    case 1: hipLaunchKernelGGL(k_extrapolate<1>, grid, dim3(256), 0, st, u, hs, kept, n, lo); break;
    case 2: hipLaunchKernelGGL(k_extrapolate<2>, grid, dim3(256), 0, st, u, hs, kept, n, lo); break;
    case 3: hipLaunchKernelGGL(k_extrapolate<3>, grid, dim3(256), 0, st, u, hs, kept, n, lo); break;
    default: hipLaunchKernelGGL(k_extrapolate<4>, grid, dim3(256), 0, st, u, hs, kept, n, lo); break;
  }
  return hipGetLastError();
}

}  // namespace smgg
