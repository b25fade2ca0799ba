// Device-side convergence bookkeeping of the batched V-cycles: the stopping
// rule of the per-mode solves (defect relative to the zero-guess defect,
// with a floor relative to the largest mode of the same problem) and the
// list of planes that still need cycles, kept on the device so that the
// host does not have to read norms back between V-cycles.
#include "smg_internal.h"
#include "vec.h"

namespace {

constexpr int kConvThreads = 1024;
constexpr int kPerThread = 4;      // list capacity kConvThreads * kPerThread
constexpr int kMaxProblems = 256;  // problems one batch can hold

// Exclusive prefix sum over the block of one int per thread (wave shuffles,
// then the wave totals); returns the thread's offset and the block total.
__device__ int block_scan(int v, int* wsum, int* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int x = v;
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  int before = 0, all = 0;
  for (int k = 0; k < nw; ++k) {
    before += k < w ? wsum[k] : 0;
    all += wsum[k];
  }
  *total = all;
  return before + x - v;
}

__device__ double sum_partial(const double* partial, int p, int nblk) {
  const auto pp = gbl(partial + (size_t)p * nblk);
  double s = 0.0;
  // 32 partials per round of loads (64 blocks per plane: two rounds), summed
  // in order
#pragma unroll 32
  for (int b = 0; b < nblk; ++b) s += pp[b];
  return sqrt(s);
}

// s_nrm[p] = sqrt(sum of the partials of list position p) for p < n: one
// position per thread, strided over the block (independent loads in flight)
__device__ void norms_to_lds(const double* partial, int n, int nblk, double* s_nrm) {
  for (int p = threadIdx.x; p < n; p += blockDim.x) s_nrm[p] = sum_partial(partial, p, nblk);
  __syncthreads();
}

__global__ void __launch_bounds__(kConvThreads) k_conv_init(const NormJob* __restrict__ jobs, const int* __restrict__ all,
                                                           int n, int n_prob, const double* __restrict__ partial,
                                                           int nblk, double tol, double floor_factor, ConvState cs,
                                                           int* __restrict__ list, int* __restrict__ count) {
  __shared__ unsigned long long dmax[kMaxProblems];
  __shared__ int buf[kConvThreads / 64];
  __shared__ double s_nrm[kConvThreads * kPerThread];
  int total;
  for (int q = threadIdx.x; q < n_prob; q += blockDim.x) dmax[q] = 0ull;
  norms_to_lds(partial, n, nblk, s_nrm);
  // the thread's entries, then their plane indices, each read for all of
  // its entries at once (indices clamped to a valid entry)
  int e[kPerThread], g[kPerThread];
  double d[kPerThread];
  const int last = max(n - 1, 0);
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) e[k] = all[min((int)threadIdx.x * kPerThread + k, last)];
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) g[k] = jobs[ent_prob(e[k])].base + ent_slot(e[k]);
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    const int p = threadIdx.x * kPerThread + k;
    if (p >= n) {
      e[k] = -1;
      continue;
    }
    const int q = ent_prob(e[k]);
    d[k] = s_nrm[p];
    gbl(cs.d0)[g[k]] = d[k];
    gbl(cs.cur)[g[k]] = d[k];
    gbl(cs.cyc)[g[k]] = 0;
    // non-negative doubles order like their bit patterns
    atomicMax(&dmax[q], (unsigned long long)__double_as_longlong(d[k]));
  }
  __syncthreads();
  int keep = 0;
  bool kk[kPerThread];
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    kk[k] = false;
    if (e[k] < 0) continue;
    const double mx = __longlong_as_double((long long)dmax[ent_prob(e[k])]);
    const double thr = tol * fmax(d[k], floor_factor * mx);
    gbl(cs.thr)[g[k]] = thr;
    kk[k] = d[k] > thr;
    keep += kk[k] ? 1 : 0;
  }
  int off = block_scan(keep, buf, &total);
#pragma unroll
  for (int k = 0; k < kPerThread; ++k)
    if (kk[k]) list[off++] = e[k];
  if (threadIdx.x == 0) *count = total;
}

__global__ void __launch_bounds__(kConvThreads) k_converge(const NormJob* __restrict__ jobs, int cap,
                                                          const double* __restrict__ partial, int nblk, ConvState cs,
                                                          int max_cycles, int count_cycle, int* __restrict__ list,
                                                          int* __restrict__ count) {
  __shared__ int buf[kConvThreads / 64];
  __shared__ double s_nrm[kConvThreads * kPerThread];
  int total;
  const int n = *count;  // every thread reads it before the block writes it
  norms_to_lds(partial, min(n, cap), nblk, s_nrm);
  // the thread's list entries, their planes' state and thresholds, each
  // kind read for all of the thread's entries at once: a position past the
  // list's end reads a position inside the buffer (clamped) and then takes
  // entry 0 (problem 0, slot 0) in its place, since the buffer need not hold
  // an entry there, so every index below is valid; nothing read for such a
  // position is used
  int e[kPerThread], g[kPerThread], c[kPerThread];
  double thr[kPerThread];
  bool kk[kPerThread];
  const int last = max(n - 1, 0);
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    const int p = (int)threadIdx.x * kPerThread + k;
    const int v = list[min(p, last)];
    e[k] = p < n ? v : 0;
  }
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) g[k] = jobs[ent_prob(e[k])].base + ent_slot(e[k]);
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    c[k] = gbl(cs.cyc)[g[k]];
    thr[k] = gbl(cs.thr)[g[k]];
  }
  int keep = 0;
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    const int p = threadIdx.x * kPerThread + k;
    kk[k] = false;
    if (p >= n) {
      e[k] = -1;
      continue;
    }
    if (p < cap) {
      const double nrm = s_nrm[p];
      gbl(cs.cur)[g[k]] = nrm;
      const int cn = c[k] + count_cycle;
      gbl(cs.cyc)[g[k]] = cn;
      kk[k] = !(nrm <= thr[k]) && cn < max_cycles;
    } else {
      kk[k] = true;  // not cycled this time
    }
    keep += kk[k] ? 1 : 0;
  }
  int off = block_scan(keep, buf, &total);  // contains a barrier: all list reads are done
#pragma unroll
  for (int k = 0; k < kPerThread; ++k)
    if (kk[k]) list[off++] = e[k];
  if (threadIdx.x == 0) *count = total;
}

}  // namespace

namespace smgk {

hipError_t mg_conv_init(const NormJob* jobs, const int* all, int n, int n_prob, const double* partial, int nblk,
                        double tol, double floor_factor, ConvState cs, int* list, int* count, hipStream_t st) {
  if (n > kConvThreads * kPerThread || n_prob > kMaxProblems || n_prob < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_conv_init, dim3(1), dim3(kConvThreads), 0, st, jobs, all, n, n_prob, partial, nblk, tol,
                     floor_factor, cs, list, count);
  return hipGetLastError();
}

hipError_t mg_converge(const NormJob* jobs, int cap, const double* partial, int nblk, ConvState cs, int max_cycles,
                       int count_cycle, int* list, int* count, hipStream_t st) {
  hipLaunchKernelGGL(k_converge, dim3(1), dim3(kConvThreads), 0, st, jobs, cap, partial, nblk, cs, max_cycles,
                     count_cycle, list, count);
  return hipGetLastError();
}

}  // namespace smgk
