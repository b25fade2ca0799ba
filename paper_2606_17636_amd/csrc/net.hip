// Kernels of the learned initial guess: a U-Net on real mode planes with
// BF16 weights and activations and FP32 accumulation on the matrix cores
// (v_mfma_f32_32x32x16_bf16 of gfx950), its backward pass and an Adam update.
//
// Activations are NHWC (pixel-major, channels contiguous) BF16 arrays; a
// 3x3 weight tensor is [c_out][9][c_in] with tap t = 3 (dy + 1) + (dx + 1)
// reading input pixel (y + dy, x + dx), zero outside the image.  A 3x3
// convolution is a GEMM with M = pixels, N = output channels and
// K = 9 c_in (k = t c_in + c), computed on LDS-staged tiles (k_conv3).  The
// weight gradient is the GEMM with M = output channels, N = k, K = pixels,
// reduced over pixel chunks (k_wgrad, k_reduce_chunks).
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

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// gfx950 matrix core: D (32 x 32, FP32) += A (32 x 16) B (16 x 32), BF16
// operands; lane l supplies A[l % 32][8 (l / 32) .. + 7] and
// B[8 (l / 32) .. + 7][l % 32]; D as in mfma_row.
__device__ __forceinline__ f32x16 mma16(uint4 a, uint4 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0, 0,
                                                 0);
}

// 3x3 convolution as a GEMM on LDS-staged tiles:
//   out[n, y, x, o] = act(b[o] + sum_{t, c} W[o, t, c] in[n, y + dy_t, x + dx_t, c]),
// optionally multiplied by (mask > 0).  A block of 4 waves computes an
// output tile of TH = 4 R rows x 32 pixels x 32 output channels: its input
// tile (TH + 2 rows x 34 pixels x CIN channels, zero outside the image) and
// the 32 x 9 CIN weights are staged in LDS once with 16-byte loads, so the
// 9 taps reuse them; each wave owns R rows and steps K = 9 CIN in slices of
// 16 (one 16-byte LDS read per operand per lane: 8 channels of one tap).
// Every thread issues all of its staging loads (addresses clamped into the
// arrays, values outside the image zeroed afterwards) before its first LDS
// store, so a block waits for one round of memory latency.
// Fused forms (ConvArgs): the decoder's concatenated input read straight
// from the level below (channels 0..31 upsampled from `lo`) and the skip
// half; the 2x2 average pooling of the output (the next level's input) and
// the 1x1 output layer computed from the tile's BF16 outputs in the same
// order as their own kernels (so the bits do not depend on the fusion).
// Grid (ceil(W / 32), ceil(H / TH), N * cout / 32).
struct ConvArgs {
  const unsigned short* in;  // input, ics elements per pixel (16-byte aligned)
  const unsigned short* lo;  // concatenated form: channels 0..31 from this (H/2 x W/2, 32 per pixel), or null
  const unsigned short* W;   // [cout][9][CIN]
  const float* bias;         // [cout] or null
  unsigned short* out;       // output, ocs per pixel, or null
  const unsigned short* mask;
  unsigned short* pooled;    // 2x2 average of the output (H/2 x W/2, pcs per pixel), or null
  const unsigned short* w1;  // 1x1 output layer weights [32] and bias, or null
  const float* b1;
  float* y1;                 // its output [N][H][W]
  int ics, ocs, mcs, pcs, cout, relu, H, Wd;
};

template <int CIN, int R>
__global__ void __launch_bounds__(256) k_conv3(const ConvArgs A) {
  constexpr int TH = 4 * R, TW = 32, K = 9 * CIN, KS = (K + 15) / 16;
  constexpr int PS = CIN + 8;       // LDS elements per staged pixel (padding spreads the lanes over banks)
  constexpr int WS = 16 * KS + 8;   // LDS elements per staged weight row
  constexpr int C8 = CIN / 8;
  constexpr int NX = (TH + 2) * (TW + 2) * C8, NXT = (NX + 255) / 256;
  constexpr int NW = 32 * (K / 8), NWT = (NW + 255) / 256;
  extern __shared__ uint4 smem_conv[];
  unsigned short* xs = reinterpret_cast<unsigned short*>(smem_conv);   // (TH + 2) * (TW + 2) * PS
  unsigned short* ws = xs + (TH + 2) * (TW + 2) * PS;                  // 32 * WS
  const int H = A.H, Wd = A.Wd;
  const int ntile = A.cout >> 5;
  const int n = blockIdx.z / ntile, ct = blockIdx.z - n * ntile;
  const int x0 = blockIdx.x * TW, y0 = blockIdx.y * TH;
  const int tid = threadIdx.x;
  uint4 wv[NWT], xv[NXT];
  unsigned inside = 0;
#pragma unroll
  for (int r = 0; r < NWT; ++r) {
    const int e = min(tid + 256 * r, NW - 1);
    const int j = e / (K / 8), q = e - j * (K / 8);
    wv[r] = *reinterpret_cast<const uint4*>(A.W + (size_t)(ct * 32 + j) * K + 8 * q);
  }
#pragma unroll
  for (int r = 0; r < NXT; ++r) {
    const int e = min(tid + 256 * r, NX - 1);
    const int q = e % C8, pix = e / C8;
    const int row = pix / (TW + 2), col = pix - row * (TW + 2);
    const int yy = y0 - 1 + row, xx = x0 - 1 + col;
    if (yy >= 0 && yy < H && xx >= 0 && xx < Wd) inside |= 1u << r;
    const int yc = min(max(yy, 0), H - 1), xc = min(max(xx, 0), Wd - 1);
    const unsigned short* src =
        (A.lo && q < 4) ? A.lo + ((size_t)(n * (H >> 1) + (yc >> 1)) * (Wd >> 1) + (xc >> 1)) * 32 + 8 * q
                        : A.in + ((size_t)(n * H + yc) * Wd + xc) * A.ics + 8 * q;
    xv[r] = *reinterpret_cast<const uint4*>(src);
  }
#pragma unroll
  for (int r = 0; r < NWT; ++r) {
    const int e = tid + 256 * r;
    if (e < NW) {
      const int j = e / (K / 8), q = e - j * (K / 8);
      *reinterpret_cast<uint4*>(ws + j * WS + 8 * q) = wv[r];
    }
  }
  if (16 * KS > K)
    for (int j = tid; j < 32; j += 256) *reinterpret_cast<uint4*>(ws + j * WS + K) = make_uint4(0, 0, 0, 0);
#pragma unroll
  for (int r = 0; r < NXT; ++r) {
    const int e = tid + 256 * r;
    if (e < NX) {
      const int q = e % C8, pix = e / C8;
      *reinterpret_cast<uint4*>(xs + pix * PS + 8 * q) = ((inside >> r) & 1u) ? xv[r] : make_uint4(0, 0, 0, 0);
    }
  }
  __syncthreads();
  const int wave = tid >> 6, lane = tid & 63;
  const int i = lane & 31, kg = lane >> 5;
  f32x16 acc[R];
  for (int r = 0; r < R; ++r)
    for (int q = 0; q < 16; ++q) acc[r][q] = 0.f;
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    const int k0 = 16 * s + 8 * kg;        // this lane's 8 k: one tap, 8 channels
    const int tap = k0 / CIN, c = k0 - tap * CIN;
    const int dy = tap / 3, dx = tap - 3 * dy;
    const uint4 b = *reinterpret_cast<const uint4*>(ws + i * WS + k0);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      uint4 a = make_uint4(0, 0, 0, 0);
      if (tap < 9) a = *reinterpret_cast<const uint4*>(xs + ((wave * R + r + dy) * (TW + 2) + i + dx) * PS + c);
      acc[r] = mma16(a, b, acc[r]);
    }
  }
  const int co = ct * 32 + i;
  const float bv = A.bias ? A.bias[co] : 0.f;
  const bool post = A.pooled || A.w1;
  unsigned short* os = xs;   // TH x TW x 32 BF16 outputs for the fused pooling / output layer
  if (post) __syncthreads();  // every wave is done reading the staged tiles
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int yl = wave * R + r, y = y0 + yl;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int xl = mfma_row(q, lane), xo = x0 + xl;
      float v = acc[r][q] + bv;
      if (A.relu) v = fmaxf(v, 0.f);
      const bool in_img = y < H && xo < Wd;
      const size_t pix = (size_t)(n * H + min(y, H - 1)) * Wd + min(xo, Wd - 1);
      if (A.mask && in_img && !(bf2f(A.mask[pix * A.mcs + co]) > 0.f)) v = 0.f;
      const unsigned short h = f2bf(v);
      if (A.out && in_img) A.out[pix * A.ocs + co] = h;
      if (post) os[(yl * TW + xl) * 32 + i] = h;
    }
  }
  if (!post) return;
  __syncthreads();
  if (A.pooled) {
    const int Hp = H >> 1, Wp = Wd >> 1;
    for (int e = tid; e < (TH / 2) * (TW / 2) * 32; e += 256) {
      const int c = e & 31, pp = e >> 5, py = pp / (TW / 2), px = pp - py * (TW / 2);
      const int yo = (y0 >> 1) + py, xo = (x0 >> 1) + px;
      if (yo >= Hp || xo >= Wp) continue;
      float sum = 0.f;
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) sum += bf2f(os[((2 * py + a) * TW + 2 * px + b) * 32 + c]);
      A.pooled[((size_t)(n * Hp + yo) * Wp + xo) * A.pcs + c] = f2bf(0.25f * sum);
    }
  }
  if (A.w1)
    for (int pl = tid; pl < TH * TW; pl += 256) {
      const int yl = pl / TW, xl = pl - yl * TW, y = y0 + yl, xo = x0 + xl;
      if (y < H && xo < Wd) {
        float sum = 0.f;
        for (int c = 0; c < 32; ++c) sum = fmaf(bf2f(A.w1[c]), bf2f(os[(yl * TW + xl) * 32 + c]), sum);
        A.y1[(size_t)(n * H + y) * Wd + xo] = sum + A.b1[0];
      }
    }
}

// Weight-gradient partials of a 3x3 convolution:
//   part[chunk][o][k] = sum over the chunk's pixels p of g[p, o] im2col(x)[p, k],
// k = t CIN + c.  A block of 4 waves takes its chunk 64 pixels at a time
// (pixels enumerated over (n, y, x)): it stages g transposed ([o][pixel])
// and the im2col slice of the 64 pixels transposed ([k][pixel], zero outside
// the image) in LDS, then each wave accumulates its 32 x 32 blocks of dW
// (columns of k) over the pixels with one 16-byte LDS read per operand per
// lane.  Grid (chunks); chunk is a multiple of 64.
template <int CIN>
__global__ void __launch_bounds__(256) k_wgrad(const unsigned short* __restrict__ g, int gcs,
                                               const unsigned short* __restrict__ x, int xcs,
                                               float* __restrict__ part, int npix, int chunk, int H, int Wd) {
  constexpr int K = 9 * CIN, KT = (K + 31) / 32;   // column tiles of 32
  constexpr int NT = (KT + 3) / 4;                 // column tiles per wave
  constexpr int P = 64, PP = P + 8;                // pixels per step, LDS row stride
  constexpr int C8 = CIN / 8;
  extern __shared__ uint4 smem_wgrad[];
  unsigned short* gs = reinterpret_cast<unsigned short*>(smem_wgrad);  // 32 * PP
  unsigned short* cs = gs + 32 * PP;                                   // 32 * KT * PP
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int i = lane & 31, kg = lane >> 5;
  const int HW = H * Wd;
  f32x16 acc[NT];
  for (int u = 0; u < NT; ++u)
    for (int q = 0; q < 16; ++q) acc[u][q] = 0.f;
  // columns beyond K stay zero
  for (int e = tid; e < (32 * KT - K) * PP; e += 256) cs[K * PP + e] = 0;
  const int p_begin = blockIdx.x * chunk, p_end = min(p_begin + chunk, npix);
  for (int p0 = p_begin; p0 < p_end; p0 += P) {
    __syncthreads();
    // g: 64 pixels x 32 channels, 16-byte loads, stored transposed
    for (int e = tid; e < P * 4; e += 256) {
      const int pl = e >> 2, q = e & 3, p = p0 + pl;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (p < p_end) v = *reinterpret_cast<const uint4*>(g + (size_t)p * gcs + 8 * q);
      const unsigned short* h = reinterpret_cast<const unsigned short*>(&v);
#pragma unroll
      for (int u = 0; u < 8; ++u) gs[(8 * q + u) * PP + pl] = h[u];
    }
    // im2col: pixel x tap, CIN channels each, stored transposed
    for (int e = tid; e < P * 9 * C8; e += 256) {
      const int q = e % C8, rest = e / C8, t = rest % 9, pl = rest / 9, p = p0 + pl;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (p < p_end) {
        const int nimg = p / HW, rem = p - nimg * HW, y = rem / Wd, xx = rem - y * Wd;
        const int yy = y + t / 3 - 1, xs_ = xx + t % 3 - 1;
        if (yy >= 0 && yy < H && xs_ >= 0 && xs_ < Wd)
          v = *reinterpret_cast<const uint4*>(x + ((size_t)(nimg * H + yy) * Wd + xs_) * xcs + 8 * q);
      }
      const unsigned short* h = reinterpret_cast<const unsigned short*>(&v);
#pragma unroll
      for (int u = 0; u < 8; ++u) cs[(t * CIN + 8 * q + u) * PP + pl] = h[u];
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < P / 16; ++s) {
      const int pk = 16 * s + 8 * kg;
      const uint4 a = *reinterpret_cast<const uint4*>(gs + i * PP + pk);
#pragma unroll
      for (int u = 0; u < NT; ++u) {
        const int tcol = wave + 4 * u;
        if (tcol < KT) {
          const uint4 b = *reinterpret_cast<const uint4*>(cs + (tcol * 32 + i) * PP + pk);
          acc[u] = mma16(a, b, acc[u]);
        }
      }
    }
  }
  // D[row = o][col = k]: lane holds column i of its tile, rows from mfma_row
  float* base = part + (size_t)blockIdx.x * 32 * K;
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    const int kc = (wave + 4 * u) * 32 + i;
    if (wave + 4 * u >= KT || kc >= K) continue;
#pragma unroll
    for (int q = 0; q < 16; ++q) base[(size_t)mfma_row(q, lane) * K + kc] = acc[u][q];
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

template <int CIN, int R>
static void launch_conv3(const ConvArgs& A, int N, hipStream_t st) {
  constexpr int KS = (9 * CIN + 15) / 16;
  constexpr size_t lds = sizeof(unsigned short) * ((4 * R + 2) * 34 * (CIN + 8) + 32 * (16 * KS + 8));
  static_assert(lds >= sizeof(unsigned short) * 4 * R * 32 * 32, "the fused post-operations reuse the staging LDS");
  dim3 grid((A.Wd + 31) / 32, (A.H + 4 * R - 1) / (4 * R), N * (A.cout / 32));
  hipLaunchKernelGGL((k_conv3<CIN, R>), grid, dim3(256), lds, st, A);
}

hipError_t conv3x(const ConvIn& I, const ConvOut& O, int N, int H, int Wd, hipStream_t st) {
  ConvArgs A{};
  A.in = I.in; A.lo = I.lo; A.W = I.W; A.bias = I.bias; A.ics = I.ics;
  A.out = O.out; A.ocs = O.ocs; A.cout = O.cout; A.mask = O.mask; A.mcs = O.mcs; A.relu = O.relu ? 1 : 0;
  A.pooled = O.pooled; A.pcs = O.pcs; A.w1 = O.w1; A.b1 = O.b1; A.y1 = O.y1;
  A.H = H; A.Wd = Wd;
  const bool post = O.pooled || O.w1;
  if (O.cout % 32 || I.ics % 8 || (reinterpret_cast<uintptr_t>(I.in) & 15)) return hipErrorInvalidValue;
  if (I.lo && (I.cin != 64 || (H & 1) || (Wd & 1) || (reinterpret_cast<uintptr_t>(I.lo) & 15))) return hipErrorInvalidValue;
  if (post && (O.cout != 32 || I.cin == 64 || (O.pooled && ((H & 1) || (Wd & 1))))) return hipErrorInvalidValue;
  switch (I.cin) {
    case 8: launch_conv3<8, 2>(A, N, st); break;
    case 32: launch_conv3<32, 2>(A, N, st); break;
    case 64: launch_conv3<64, 1>(A, N, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t conv3(const unsigned short* in, int ics, int cin, const unsigned short* W, const float* bias,
                 unsigned short* out, int ocs, int cout, const unsigned short* mask, int mcs, bool relu, int N, int H,
                 int Wd, hipStream_t st) {
  ConvIn I{in, nullptr, ics, cin, W, bias};
  ConvOut O{out, ocs, cout, mask, mcs, relu, nullptr, 0, nullptr, nullptr, nullptr};
  return conv3x(I, O, N, H, Wd, st);
}

int wgrad_chunk(int npix, int cout, int cin) {
  const size_t K = 9 * (size_t)cin;
  int chunk = 1024;
  while ((size_t)((npix + chunk - 1) / chunk) * cout * K > kWgradMaxPartials) chunk *= 2;
  return chunk;
}

size_t wgrad_partials(int npix, int cout, int cin) {
  const int chunk = wgrad_chunk(npix, cout, cin);
  return (size_t)((npix + chunk - 1) / chunk) * cout * 9 * cin;
}

hipError_t wgrad(const unsigned short* g, int gcs, int cout, const unsigned short* x, int xcs, int cin, float* part,
                 size_t part_floats, float* dW, float* db, int N, int H, int Wd, hipStream_t st) {
  if (cout != 32 || gcs % 8 || xcs % 8) return hipErrorInvalidValue;
  const int npix = N * H * Wd, K = 9 * cin;
  const int chunk = wgrad_chunk(npix, cout, cin);
  const int nchunk = (npix + chunk - 1) / chunk;
  if ((size_t)nchunk * cout * K > part_floats) return hipErrorInvalidValue;
  // LDS: g (32 rows) and the im2col slice (32 KT rows), 72 elements each
  const size_t lds = sizeof(unsigned short) * 72 * (32 + 32 * ((K + 31) / 32));
  switch (cin) {
    case 8: hipLaunchKernelGGL(k_wgrad<8>, dim3(nchunk), dim3(256), lds, st, g, gcs, x, xcs, part, npix, chunk, H, Wd); break;
    case 32: hipLaunchKernelGGL(k_wgrad<32>, dim3(nchunk), dim3(256), lds, st, g, gcs, x, xcs, part, npix, chunk, H, Wd); break;
    case 64: hipLaunchKernelGGL(k_wgrad<64>, dim3(nchunk), dim3(256), lds, st, g, gcs, x, xcs, part, npix, chunk, H, Wd); break;
    default: return hipErrorInvalidValue;
  }
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
