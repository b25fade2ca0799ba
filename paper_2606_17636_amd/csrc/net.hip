// Kernels of the learned initial guess: a U-Net on real mode planes with
// BF16 weights and activations and FP32 accumulation on the matrix cores
// (v_mfma_f32_32x32x8_bf16), its backward pass and an Adam update.
//
// Activations are NHWC (pixel-major, channels contiguous) BF16 arrays; a
// 3x3 weight tensor is [c_out][9][c_in] with tap t = 3 (dy + 1) + (dx + 1)
// reading input pixel (y + dy, x + dx), zero outside the image.  A 3x3
// convolution is a GEMM with M = pixels, N = output channels and
// K = 9 c_in (k = t c_in + c): one wave computes 32 pixels of one image row
// times 32 output channels, each lane feeding four consecutive k of its
// pixel (one tap, four channels: one 8-byte load) and four of its output
// channel's weights.  The weight gradient is the GEMM with M = output
// channels, N = k, K = pixels, reduced over pixel chunks.
#include <hip/hip_runtime.h>

#include "net_internal.h"

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ unsigned short f2bf(float x) {
  unsigned u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return (unsigned short)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest, ties to even
  return (unsigned short)(u >> 16);
}

__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float(((unsigned)h) << 16); }

// D layout of the 32x32x8 MFMA: register r of lane l holds row
// 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32.
__device__ __forceinline__ int mfma_row(int r, int lane) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

// out[n, y, x, o] = act(b[o] + sum_{t, c} W[o, t, c] in[n, y + dy_t, x + dx_t, c]),
// optionally multiplied by (mask > 0).  Grid (ceil(W/32), H, N * cout/32),
// one wave per block.  cin % 4 == 0, cout % 32 == 0; channel strides and
// base pointers select sub-ranges of wider (concatenated) arrays.
__global__ void __launch_bounds__(64) k_conv3(const unsigned short* __restrict__ in, int ics, int cin,
                                             const unsigned short* __restrict__ Wt, const float* __restrict__ bias,
                                             unsigned short* __restrict__ out, int ocs, int cout,
                                             const unsigned short* __restrict__ mask, int mcs, int relu, int H, int Wd) {
  const int lane = threadIdx.x;
  const int x0 = blockIdx.x * 32, y = blockIdx.y;
  const int ntile = cout >> 5;
  const int n = blockIdx.z / ntile, ct = blockIdx.z - n * ntile;
  const int i = lane & 31, kg = lane >> 5;
  const int px = x0 + i;
  const int K = 9 * cin;
  const unsigned short* wrow = Wt + (size_t)(ct * 32 + i) * K;
  f32x16 acc;
  for (int r = 0; r < 16; ++r) acc[r] = 0.f;
  for (int k0 = 0; k0 < K; k0 += 8) {
    const int k = k0 + 4 * kg;
    bf16x4 a = {0, 0, 0, 0}, b = {0, 0, 0, 0};
    if (k < K) {
      const int tap = k / cin, c = k - tap * cin;
      const int yy = y + tap / 3 - 1, xx = px + tap % 3 - 1;
      if (yy >= 0 && yy < H && xx >= 0 && xx < Wd)
        a = *reinterpret_cast<const bf16x4*>(in + ((size_t)(n * H + yy) * Wd + xx) * ics + c);
      b = *reinterpret_cast<const bf16x4*>(wrow + k);
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
  }
  const int co = ct * 32 + i;
  const float bv = bias ? bias[co] : 0.f;
  for (int r = 0; r < 16; ++r) {
    const int xo = x0 + mfma_row(r, lane);
    if (xo >= Wd) continue;
    float v = acc[r] + bv;
    if (relu) v = fmaxf(v, 0.f);
    const size_t pix = (size_t)(n * H + y) * Wd + xo;
    if (mask && !(bf2f(mask[pix * mcs + co]) > 0.f)) v = 0.f;
    out[pix * ocs + co] = f2bf(v);
  }
}

// Weight gradient partials: part[chunk][o][k] = sum over the chunk's pixels
// of g[p, o] * im2col(x)[p, k].  Grid (ceil(K/32), cout/32, chunks), one
// wave per block; pixels are enumerated over (n, y, x).
__global__ void __launch_bounds__(64) k_wgrad(const unsigned short* __restrict__ g, int gcs, int cout,
                                             const unsigned short* __restrict__ x, int xcs, int cin,
                                             float* __restrict__ part, int npix, int chunk, int H, int Wd) {
  const int lane = threadIdx.x;
  const int i = lane & 31, kg = lane >> 5;
  const int K = 9 * cin;
  const int kcol = blockIdx.x * 32 + i;  // this lane's B column (k)
  const int o = blockIdx.y * 32 + i;     // this lane's A row (output channel)
  int tap = 0, c = 0;
  const bool kin = kcol < K;
  if (kin) { tap = kcol / cin; c = kcol - tap * cin; }
  const int dy = tap / 3 - 1, dx = tap % 3 - 1;
  const int p0 = blockIdx.z * chunk, p1 = min(p0 + chunk, npix);
  const int HW = H * Wd;
  f32x16 acc;
  for (int r = 0; r < 16; ++r) acc[r] = 0.f;
  for (int pb = p0; pb < p1; pb += 8) {
    bf16x4 a, b;
    for (int v = 0; v < 4; ++v) {
      const int p = pb + 4 * kg + v;
      unsigned short av = 0, bv = 0;
      if (p < p1) {
        av = g[(size_t)p * gcs + o];
        if (kin) {
          const int n = p / HW, rem = p - n * HW, yy = rem / Wd + dy, xx = rem % Wd + dx;
          if (yy >= 0 && yy < H && xx >= 0 && xx < Wd) bv = x[((size_t)(n * H + yy) * Wd + xx) * xcs + c];
        }
      }
      a[v] = (short)av;
      b[v] = (short)bv;
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
  }
  // D[row = o local][col = k local]: lane holds column i (k), rows from mfma_row
  const size_t base = (size_t)blockIdx.z * cout * K;
  for (int r = 0; r < 16; ++r) {
    const int orow = blockIdx.y * 32 + mfma_row(r, lane);
    if (kin) part[base + (size_t)orow * K + kcol] = acc[r];
  }
}

// dW[j] = sum over chunks of part[chunk][j]
__global__ void k_reduce_chunks(const float* __restrict__ part, int nchunk, int len, float* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= len) return;
  float s = 0.f;
  for (int q = 0; q < nchunk; ++q) s += part[(size_t)q * len + j];
  out[j] = s;
}

// db[o] += sum over pixels of g[p, o] (one block per pixel chunk; block 256)
__global__ void k_bias_grad(const unsigned short* __restrict__ g, int gcs, int cout, int npix, int chunk,
                            float* __restrict__ db) {
  __shared__ float red[256];
  const int o = threadIdx.x % cout, lane_p = threadIdx.x / cout, ppb = blockDim.x / cout;
  const int p0 = blockIdx.x * chunk, p1 = min(p0 + chunk, npix);
  float s = 0.f;
  for (int p = p0 + lane_p; p < p1; p += ppb) s += bf2f(g[(size_t)p * gcs + o]);
  red[threadIdx.x] = s;
  __syncthreads();
  if (lane_p == 0) {
    float t = 0.f;
    for (int k = 0; k < ppb; ++k) t += red[k * cout + o];
    atomicAdd(&db[o], t);
  }
}

// Weights of the data gradient: Wd[c][t][o] = W[o][8 - t][c]
__global__ void k_flip_weights(const unsigned short* __restrict__ W, int cout, int cin, unsigned short* __restrict__ Wd) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int total = cout * 9 * cin;
  if (idx >= total) return;
  const int o = idx / (9 * cin), rem = idx - o * 9 * cin, t = rem / cin, c = rem - t * cin;
  Wd[((size_t)c * 9 + (8 - t)) * cout + o] = W[idx];
}

// 2x2 average pooling: out (H/2, W/2) <- in (H, W), rounded to BF16
__global__ void k_pool(const unsigned short* __restrict__ in, int ics, unsigned short* __restrict__ out, int ocs, int C,
                       int N, int H, int Wd) {
  const int Ho = H / 2, Wo = Wd / 2;
  const size_t total = (size_t)N * Ho * Wo * C;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(t % C);
    const size_t pix = t / C;
    const int xo = (int)(pix % Wo), yo = (int)((pix / Wo) % Ho), n = (int)(pix / ((size_t)Wo * Ho));
    float s = 0.f;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) s += bf2f(in[((size_t)(n * H + 2 * yo + a) * Wd + 2 * xo + b) * ics + c]);
    out[pix * ocs + c] = f2bf(0.25f * s);
  }
}

// nearest upsampling by 2: out (2H, 2W) <- in (H, W)
__global__ void k_up(const unsigned short* __restrict__ in, int ics, unsigned short* __restrict__ out, int ocs, int C, int N,
                     int H, int Wd) {
  const int Ho = 2 * H, Wo = 2 * Wd;
  const size_t total = (size_t)N * Ho * Wo * C;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(t % C);
    const size_t pix = t / C;
    const int xo = (int)(pix % Wo), yo = (int)((pix / Wo) % Ho), n = (int)(pix / ((size_t)Wo * Ho));
    out[pix * ocs + c] = in[((size_t)(n * H + yo / 2) * Wd + xo / 2) * ics + c];
  }
}

// gradient through the upsampling: gout (H, W) = bf16(sum of the 4 children
// of gin (2H, 2W)) * (mask > 0)
__global__ void k_up_back(const unsigned short* __restrict__ gin, int gcs, const unsigned short* __restrict__ mask,
                          int mcs, unsigned short* __restrict__ gout, int ocs, int C, int N, int H, int Wd) {
  const size_t total = (size_t)N * H * Wd * C;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(t % C);
    const size_t pix = t / C;
    const int x = (int)(pix % Wd), y = (int)((pix / Wd) % H), n = (int)(pix / ((size_t)Wd * H));
    float s = 0.f;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) s += bf2f(gin[((size_t)(n * 2 * H + 2 * y + a) * 2 * Wd + 2 * x + b) * gcs + c]);
    if (!(bf2f(mask[pix * mcs + c]) > 0.f)) s = 0.f;
    gout[pix * ocs + c] = f2bf(s);
  }
}

// gradient into an encoder output e (H, W): bf16((bf16(gpool / 4) + skip) * (e > 0))
// with gpool the gradient of the pooled level (H/2, W/2)
__global__ void k_pool_back(const unsigned short* __restrict__ gpool, int pcs, const unsigned short* __restrict__ skip,
                            int scs, const unsigned short* __restrict__ e, int ecs, unsigned short* __restrict__ gout,
                            int ocs, int C, int N, int H, int Wd) {
  const size_t total = (size_t)N * H * Wd * C;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(t % C);
    const size_t pix = t / C;
    const int x = (int)(pix % Wd), y = (int)((pix / Wd) % H), n = (int)(pix / ((size_t)Wd * H));
    const float gp = bf2f(f2bf(0.25f * bf2f(gpool[((size_t)(n * (H / 2) + y / 2) * (Wd / 2) + x / 2) * pcs + c])));
    float s = gp + bf2f(skip[pix * scs + c]);
    if (!(bf2f(e[pix * ecs + c]) > 0.f)) s = 0.f;
    gout[pix * ocs + c] = f2bf(s);
  }
}

// input planes (FP32 NHWC, 4 channels) -> BF16
__global__ void k_to_bf16(const float* __restrict__ in, unsigned short* __restrict__ out, size_t n) {
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x)
    out[t] = f2bf(in[t]);
}

// 1x1 output layer: y[p] = b + sum_c w[c] d[p, c]  (FP32 output)
__global__ void k_out(const unsigned short* __restrict__ d, int dcs, int C, const unsigned short* __restrict__ w,
                      const float* __restrict__ b, float* __restrict__ y, int npix) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npix) return;
  float s = 0.f;
  for (int c = 0; c < C; ++c) s = fmaf(bf2f(w[c]), bf2f(d[(size_t)p * dcs + c]), s);
  y[p] = s + b[0];
}

// backward of the output layer: gd[p, c] = bf16(gy[p] w[c]) * (d > 0);
// dw[c] += sum_p gy[p] d[p, c]; db += sum_p gy[p].  Block 256 = 8 pixels x 32 channels.
__global__ void k_out_back(const float* __restrict__ gy, const unsigned short* __restrict__ d, int dcs,
                           const unsigned short* __restrict__ w, unsigned short* __restrict__ gd, int gcs, int npix,
                           float* __restrict__ dw, float* __restrict__ db) {
  __shared__ float red[256];
  const int c = threadIdx.x & 31, pl = threadIdx.x >> 5;
  float sw = 0.f, sb = 0.f;
  for (int p = blockIdx.x * 8 + pl; p < npix; p += gridDim.x * 8) {
    const float g = gy[p];
    const float dv = bf2f(d[(size_t)p * dcs + c]);
    float v = g * bf2f(w[c]);
    if (!(dv > 0.f)) v = 0.f;
    gd[(size_t)p * gcs + c] = f2bf(v);
    sw = fmaf(g, dv, sw);
    if (c == 0) sb += g;
  }
  red[threadIdx.x] = sw;
  __syncthreads();
  if (pl == 0) {
    float t = 0.f;
    for (int k = 0; k < 8; ++k) t += red[k * 32 + c];
    atomicAdd(&dw[c], t);
  }
  __syncthreads();
  red[threadIdx.x] = c == 0 ? sb : 0.f;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.f;
    for (int k = 0; k < 8; ++k) t += red[k * 32];
    atomicAdd(db, t);
  }
}

// mean squared error: loss += sum (y - t)^2 / n; gy = 2 (y - t) / n
__global__ void k_mse(const float* __restrict__ y, const float* __restrict__ tgt, float* __restrict__ gy, int n,
                      float* __restrict__ loss) {
  __shared__ float red[256];
  float s = 0.f;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
    const float d = y[p] - tgt[p];
    gy[p] = 2.f * d / (float)n;
    s += d * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(loss, red[0] / (float)n);
}

// Adam on the FP32 master parameters, then their BF16 copy
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       unsigned short* __restrict__ pb, int n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[i] = pi;
  pb[i] = f2bf(pi);
}

__global__ void k_params_bf16(const float* __restrict__ p, unsigned short* __restrict__ pb, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) pb[i] = f2bf(p[i]);
}

__global__ void k_fill_f32(float* __restrict__ p, size_t n, float v) {
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) p[t] = v;
}

unsigned grid1(size_t n, unsigned block = 256) {
  size_t g = (n + block - 1) / block;
  if (g > 65535) g = 65535;
  return (unsigned)(g ? g : 1);
}

}  // namespace

namespace smgn {

hipError_t conv3(const unsigned short* in, int ics, int cin, const unsigned short* W, const float* bias,
                 unsigned short* out, int ocs, int cout, const unsigned short* mask, int mcs, bool relu, int N, int H,
                 int Wd, hipStream_t st) {
  if (cin % 4 || cout % 32 || ics % 4) return hipErrorInvalidValue;
  dim3 grid((Wd + 31) / 32, H, N * (cout / 32));
  hipLaunchKernelGGL(k_conv3, grid, dim3(64), 0, st, in, ics, cin, W, bias, out, ocs, cout, mask, mcs, relu ? 1 : 0, H,
                     Wd);
  return hipGetLastError();
}

hipError_t wgrad(const unsigned short* g, int gcs, int cout, const unsigned short* x, int xcs, int cin, float* part,
                 size_t part_floats, float* dW, float* db, int N, int H, int Wd, hipStream_t st) {
  if (cout % 32) return hipErrorInvalidValue;
  const int npix = N * H * Wd, K = 9 * cin;
  int chunk = 1024;
  int nchunk = (npix + chunk - 1) / chunk;
  while ((size_t)nchunk * cout * K > part_floats) {
    chunk *= 2;
    nchunk = (npix + chunk - 1) / chunk;
  }
  dim3 grid((K + 31) / 32, cout / 32, nchunk);
  hipLaunchKernelGGL(k_wgrad, grid, dim3(64), 0, st, g, gcs, cout, x, xcs, cin, part, npix, chunk, H, Wd);
  const int len = cout * K;
  hipLaunchKernelGGL(k_reduce_chunks, dim3((len + 255) / 256), dim3(256), 0, st, part, nchunk, len, dW);
  const int bchunk = 2048;
  hipLaunchKernelGGL(k_bias_grad, dim3((npix + bchunk - 1) / bchunk), dim3(256), 0, st, g, gcs, cout, npix, bchunk, db);
  return hipGetLastError();
}

hipError_t flip_weights(const unsigned short* W, int cout, int cin, unsigned short* Wd, hipStream_t st) {
  const int total = cout * 9 * cin;
  hipLaunchKernelGGL(k_flip_weights, dim3((total + 255) / 256), dim3(256), 0, st, W, cout, cin, Wd);
  return hipGetLastError();
}

hipError_t pool(const unsigned short* in, int ics, unsigned short* out, int ocs, int C, int N, int H, int Wd,
                hipStream_t st) {
  hipLaunchKernelGGL(k_pool, dim3(grid1((size_t)N * H * Wd * C / 4)), dim3(256), 0, st, in, ics, out, ocs, C, N, H, Wd);
  return hipGetLastError();
}

hipError_t up(const unsigned short* in, int ics, unsigned short* out, int ocs, int C, int N, int H, int Wd,
              hipStream_t st) {
  hipLaunchKernelGGL(k_up, dim3(grid1((size_t)N * H * Wd * C * 4)), dim3(256), 0, st, in, ics, out, ocs, C, N, H, Wd);
  return hipGetLastError();
}

hipError_t up_back(const unsigned short* gin, int gcs, const unsigned short* mask, int mcs, unsigned short* gout, int ocs,
                   int C, int N, int H, int Wd, hipStream_t st) {
  hipLaunchKernelGGL(k_up_back, dim3(grid1((size_t)N * H * Wd * C)), dim3(256), 0, st, gin, gcs, mask, mcs, gout, ocs, C,
                     N, H, Wd);
  return hipGetLastError();
}

hipError_t pool_back(const unsigned short* gpool, int pcs, const unsigned short* skip, int scs, const unsigned short* e,
                     int ecs, unsigned short* gout, int ocs, int C, int N, int H, int Wd, hipStream_t st) {
  hipLaunchKernelGGL(k_pool_back, dim3(grid1((size_t)N * H * Wd * C)), dim3(256), 0, st, gpool, pcs, skip, scs, e, ecs,
                     gout, ocs, C, N, H, Wd);
  return hipGetLastError();
}

hipError_t to_bf16(const float* in, unsigned short* out, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_to_bf16, dim3(grid1(n)), dim3(256), 0, st, in, out, n);
  return hipGetLastError();
}

hipError_t out_layer(const unsigned short* d, int dcs, int C, const unsigned short* w, const float* b, float* y, int npix,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_out, dim3((npix + 255) / 256), dim3(256), 0, st, d, dcs, C, w, b, y, npix);
  return hipGetLastError();
}

hipError_t out_layer_back(const float* gy, const unsigned short* d, int dcs, const unsigned short* w, unsigned short* gd,
                          int gcs, int npix, float* dw, float* db, hipStream_t st) {
  hipLaunchKernelGGL(k_out_back, dim3(std::min(4096, (npix + 7) / 8)), dim3(256), 0, st, gy, d, dcs, w, gd, gcs, npix, dw,
                     db);
  return hipGetLastError();
}

hipError_t mse(const float* y, const float* t, float* gy, int n, float* loss, hipStream_t st) {
  hipLaunchKernelGGL(k_mse, dim3(std::min(1024, (n + 255) / 256)), dim3(256), 0, st, y, t, gy, n, loss);
  return hipGetLastError();
}

hipError_t adam(float* p, const float* g, float* m, float* v, unsigned short* pb, int n, float lr, float b1, float b2,
                float eps, int step, hipStream_t st) {
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, st, p, g, m, v, pb, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t params_bf16(const float* p, unsigned short* pb, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_params_bf16, dim3((n + 255) / 256), dim3(256), 0, st, p, pb, n);
  return hipGetLastError();
}

hipError_t fill_f32(float* p, size_t n, float v, hipStream_t st) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f32, dim3(grid1(n)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

}  // namespace smgn
