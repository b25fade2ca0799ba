// Per-mode geometric multigrid kernels (Sec. 3), batched over planes.
//
// A level stores each plane as an interleaved complex FP64 array [na][nb]
// (b fastest).  The operator of mode m at (i, j) is
//   (L u)_ij = ua_i u_{i+1,j} + da_i u_{i-1,j} + Rr_i (ub_j u_{i,j+1} + db_j u_{i,j-1})
//            + (Ca[m]_i + Rr_i Cb[m]_j) u_ij
// with the ghost couplings already zero (boundary data live in f, ghosts that
// mirror the adjacent cell live in the diagonal), so no kernel branches on
// boundaries: out-of-range neighbours are read as zeros (LDS padding) or
// through clamped indices whose coupling is zero.
//
// Smoother (Sec. 3.2, Algorithm 1, ordering of Sec. 5.2): one launch per
// line direction.  A block owns a tile that spans whole lines plus two halo
// lines on each side across the lines; the first zebra colour is also
// computed on the inner halo line so the second colour sees the updated
// neighbours without another pass over memory.  Inside a colour the n_sor
// even-odd SOR passes of every line run as point updates in LDS.
#include "smg_internal.h"

namespace {

constexpr int kThreads = 256;

struct Cx {
  __device__ static double2 add(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
};

__device__ __forceinline__ double2 axpy(double a, double2 x, double2 y) {
  return make_double2(fma(a, x.x, y.x), fma(a, x.y, y.y));
}

// Residual f - L u at (i, j) of one plane, reading u from global memory.
__device__ __forceinline__ double2 resid_at(const LevelDev& L, int m, const double2* __restrict__ u,
                                            const double2* __restrict__ f, int i, int j) {
  const int na = L.na, nb = L.nb;
  const size_t row = (size_t)i * nb;
  const int ip = min(i + 1, na - 1), im = max(i - 1, 0);
  const int jp = min(j + 1, nb - 1), jm = max(j - 1, 0);
  const double R = L.Rr[i];
  const double c = L.Ca[(size_t)m * na + i] + R * L.Cb[(size_t)m * nb + j];
  double2 uc = u[row + j];
  double2 acc = make_double2(c * uc.x, c * uc.y);
  acc = axpy(L.ua[i], u[(size_t)ip * nb + j], acc);
  acc = axpy(L.da[i], u[(size_t)im * nb + j], acc);
  acc = axpy(R * L.ub[j], u[row + jp], acc);
  acc = axpy(R * L.db[j], u[row + jm], acc);
  double2 fv = f[row + j];
  return make_double2(fv.x - acc.x, fv.y - acc.y);
}

// ---------------------------------------------------------------------------
// Smoother.  DIR = 1: polar lines (rows i, points along j); tile = rows
// [i0-2, i0+T+2) x all columns.  DIR = 0: radial lines (columns j, points
// along i); tile = all rows x columns [j0-2, j0+W+2).  LDS holds the tile
// with one zero column/row of padding at the ends of the lines.
// ---------------------------------------------------------------------------
template <int DIR, bool EXACT>
__global__ void __launch_bounds__(kThreads) k_smooth(LevelDev L, Batch bt, double2* __restrict__ U,
                                                    const double2* __restrict__ F, int n_sor, int tile) {
  extern __shared__ double2 sh[];
  const int p = blockIdx.y;
  const int slot = bt.slot[p], m = bt.mode[p];
  const int na = L.na, nb = L.nb;
  double2* u = U + (size_t)slot * na * nb;
  const double2* f = F + (size_t)slot * na * nb;
  // tile geometry in (row, col) = (i, j) coordinates
  int r0, nr, c0, nc;  // first global row/col held in LDS and counts (incl. halo/pad)
  if (DIR == 1) {
    const int i0 = blockIdx.x * tile;
    r0 = i0 - 2; nr = tile + 4;
    c0 = -1; nc = nb + 2;
  } else {
    const int j0 = blockIdx.x * tile;
    r0 = -1; nr = na + 2;
    c0 = j0 - 2; nc = tile + 4;
  }
  // load the tile (zeros outside the plane)
  for (int t = threadIdx.x; t < nr * nc; t += blockDim.x) {
    const int rr = t / nc, cc = t - rr * nc;
    const int i = r0 + rr, j = c0 + cc;
    double2 v = make_double2(0.0, 0.0);
    if (i >= 0 && i < na && j >= 0 && j < nb) v = u[(size_t)i * nb + j];
    sh[t] = v;
  }
  __syncthreads();
  // line range of this tile (the coordinate across the lines)
  const int lbeg = blockIdx.x * tile;                     // first owned line
  const int lend = min(lbeg + tile, DIR == 1 ? na : nb);  // one past the last owned line
  const int nlines_total = DIR == 1 ? na : nb;
  const int npts = DIR == 1 ? nb : na;                    // points per line
  // scratch for the exact line solve: one row of Thomas factors per line
  double* cp = reinterpret_cast<double*>(sh + nr * nc);
  for (int lc = 0; lc < 2; ++lc) {
    // colour lc: first colour includes the inner halo lines
    int a = lc == 0 ? lbeg - 1 : lbeg;
    int b = lc == 0 ? lend + 1 : lend;  // exclusive
    a = max(a, 0);
    b = min(b, nlines_total);
    if ((a & 1) != lc) ++a;
    const int nl = a < b ? (b - a + 1) / 2 : 0;  // lines a, a+2, ... < b
    if (EXACT) {
      // Thomas algorithm along each line of the colour; the couplings to the
      // neighbouring lines (the other colour) are fixed right-hand-side terms.
      for (int t = threadIdx.x; t < nl; t += blockDim.x) {
        const int line = a + 2 * t;
        double* c1 = cp + t * npts;
        double2 prev = make_double2(0.0, 0.0);
        double cprev = 0.0;
        for (int k = 0; k < npts; ++k) {
          const int i = DIR == 1 ? line : k;
          const int j = DIR == 1 ? k : line;
          const int rr = i - r0, cc = j - c0;
          const double R = L.Rr[i];
          const double c = L.Ca[(size_t)m * na + i] + R * L.Cb[(size_t)m * nb + j];
          double lo, up;
          double2 o1, o2;
          double w1, w2;
          if (DIR == 1) {  // line along j; fixed neighbours i+1, i-1
            lo = R * L.db[j]; up = R * L.ub[j];
            o1 = sh[(rr + 1) * nc + cc]; o2 = sh[(rr - 1) * nc + cc];
            w1 = L.ua[i]; w2 = L.da[i];
          } else {         // line along i; fixed neighbours j+1, j-1
            lo = L.da[i]; up = L.ua[i];
            o1 = sh[rr * nc + cc + 1]; o2 = sh[rr * nc + cc - 1];
            w1 = R * L.ub[j]; w2 = R * L.db[j];
          }
          const double2 fv = f[(size_t)i * nb + j];
          const double rx = fv.x - (w1 * o1.x + w2 * o2.x);
          const double ry = fv.y - (w1 * o1.y + w2 * o2.y);
          const double den = c - lo * cprev;
          cprev = up / den;
          c1[k] = cprev;
          prev = make_double2((rx - lo * prev.x) / den, (ry - lo * prev.y) / den);
          sh[rr * nc + cc] = prev;
        }
        for (int k = npts - 2; k >= 0; --k) {
          const int i = DIR == 1 ? line : k;
          const int j = DIR == 1 ? k : line;
          const int rr = i - r0, cc = j - c0;
          const double2 nx = DIR == 1 ? sh[rr * nc + cc + 1] : sh[(rr + 1) * nc + cc];
          const double2 d = sh[rr * nc + cc];
          sh[rr * nc + cc] = make_double2(d.x - c1[k] * nx.x, d.y - c1[k] * nx.y);
        }
      }
      __syncthreads();
      continue;
    }
    for (int it = 0; it < n_sor; ++it) {
      for (int pc = 0; pc < 2; ++pc) {
        const int np = (npts - pc + 1) / 2;  // points pc, pc+2, ... < npts
        const int total = nl * np;
        for (int t = threadIdx.x; t < total; t += blockDim.x) {
          int line, pt;
          if (DIR == 1) {
            line = a + 2 * (t / np);
            pt = pc + 2 * (t % np);
          } else {
            pt = pc + 2 * (t / nl);
            line = a + 2 * (t % nl);
          }
          const int i = DIR == 1 ? line : pt;
          const int j = DIR == 1 ? pt : line;
          const int rr = i - r0, cc = j - c0;
          double2* me = &sh[rr * nc + cc];
          const double2 un = sh[(rr + 1) * nc + cc];
          const double2 us = sh[(rr - 1) * nc + cc];
          const double2 ue = sh[rr * nc + cc + 1];
          const double2 uw = sh[rr * nc + cc - 1];
          const double R = L.Rr[i];
          const double c = L.Ca[(size_t)m * na + i] + R * L.Cb[(size_t)m * nb + j];
          const double w = DIR == 1 ? L.wb[(size_t)m * na + i] : L.wr[(size_t)m * nb + j];
          const double ua = L.ua[i], da = L.da[i], ub = R * L.ub[j], db = R * L.db[j];
          const double2 fv = f[(size_t)i * nb + j];
          double sx = ua * un.x + da * us.x + ub * ue.x + db * uw.x;
          double sy = ua * un.y + da * us.y + ub * ue.y + db * uw.y;
          const double2 old = *me;
          const double tx = (fv.x - sx) / c, ty = (fv.y - sy) / c;
          *me = make_double2(old.x + w * (tx - old.x), old.y + w * (ty - old.y));
        }
        __syncthreads();
      }
    }
  }
  // write back the owned lines
  if (DIR == 1) {
    for (int t = threadIdx.x; t < (lend - lbeg) * nb; t += blockDim.x) {
      const int i = lbeg + t / nb, j = t % nb;
      u[(size_t)i * nb + j] = sh[(i - r0) * nc + (j - c0)];
    }
  } else {
    const int w = lend - lbeg;
    for (int t = threadIdx.x; t < na * w; t += blockDim.x) {
      const int i = t / w, j = lbeg + t % w;
      u[(size_t)i * nb + j] = sh[(i - r0) * nc + (j - c0)];
    }
  }
}

__global__ void __launch_bounds__(kThreads) k_residual(LevelDev L, Batch bt, const double2* __restrict__ U,
                                                      const double2* __restrict__ F, double2* __restrict__ Rout) {
  const int p = blockIdx.y;
  const int slot = bt.slot[p], m = bt.mode[p];
  const size_t off = (size_t)slot * L.na * L.nb;
  const int cells = L.na * L.nb;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < cells; t += gridDim.x * blockDim.x) {
    const int i = t / L.nb, j = t - i * L.nb;
    Rout[off + t] = resid_at(L, m, U + off, F + off, i, j);
  }
}

// Coarse right-hand side = bilinear restriction of the fine residual; the
// coarse correction starts from zero.
__global__ void __launch_bounds__(kThreads) k_restrict(LevelDev L, LevelDev C, Batch bt, const double2* __restrict__ U,
                                                      const double2* __restrict__ F, double2* __restrict__ FC,
                                                      double2* __restrict__ UC) {
  const int p = blockIdx.y;
  const int slot = bt.slot[p], m = bt.mode[p];
  const size_t off = (size_t)slot * L.na * L.nb;
  const size_t offc = (size_t)slot * C.na * C.nb;
  const int cells = C.na * C.nb;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < cells; t += gridDim.x * blockDim.x) {
    const int I = t / C.nb, J = t - I * C.nb;
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const double wa = L.rwa[2 * I + a];
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const double w = wa * L.rwb[2 * J + b];
        const double2 r = resid_at(L, m, U + off, F + off, 2 * I + a, 2 * J + b);
        acc = axpy(w, r, acc);
      }
    }
    FC[offc + t] = acc;
    UC[offc + t] = make_double2(0.0, 0.0);
  }
}

__global__ void __launch_bounds__(kThreads) k_prolong(LevelDev L, LevelDev C, Batch bt, double2* __restrict__ U,
                                                     const double2* __restrict__ UC) {
  const int p = blockIdx.y;
  const int slot = bt.slot[p], m = bt.mode[p];
  const size_t off = (size_t)slot * L.na * L.nb;
  const size_t offc = (size_t)slot * C.na * C.nb;
  const int par = m & 1;
  const int cells = L.na * L.nb;
  const int* pbi0 = L.pb_i0 + par * L.nb;
  const int* pbi1 = L.pb_i1 + par * L.nb;
  const double* pbw0 = L.pb_w0 + par * L.nb;
  const double* pbw1 = L.pb_w1 + par * L.nb;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < cells; t += gridDim.x * blockDim.x) {
    const int i = t / L.nb, j = t - i * L.nb;
    const int a0 = L.pa_i0[i], a1 = L.pa_i1[i];
    const int b0 = pbi0[j], b1 = pbi1[j];
    const double wa0 = L.pa_w0[i], wa1 = L.pa_w1[i];
    const double wb0 = pbw0[j], wb1 = pbw1[j];
    const double2* uc = UC + offc;
    double2 e = make_double2(0.0, 0.0);
    e = axpy(wa0 * wb0, uc[(size_t)a0 * C.nb + b0], e);
    e = axpy(wa0 * wb1, uc[(size_t)a0 * C.nb + b1], e);
    e = axpy(wa1 * wb0, uc[(size_t)a1 * C.nb + b0], e);
    e = axpy(wa1 * wb1, uc[(size_t)a1 * C.nb + b1], e);
    double2 v = U[off + t];
    U[off + t] = make_double2(v.x + e.x, v.y + e.y);
  }
}

// Coarsest level (Sec. 3.3): red-black point SOR with the 2D WKB omega from a
// zero start, one block per plane, the plane resident in LDS; stops when the
// residual 2-norm has dropped by rtol or after max_sweeps sweeps.
__global__ void __launch_bounds__(kThreads) k_coarse(LevelDev L, Batch bt, double2* __restrict__ U,
                                                    const double2* __restrict__ F, double rtol, int max_sweeps) {
  extern __shared__ double2 sh[];
  __shared__ double red[kThreads / 64];
  const int p = blockIdx.x;
  const int slot = bt.slot[p], m = bt.mode[p];
  const int na = L.na, nb = L.nb;
  const int nc = nb + 2;
  double2* us = sh;                       // (na+2) x (nb+2), zero border
  double2* fs = sh + (na + 2) * nc;       // na x nb
  const size_t off = (size_t)slot * na * nb;
  for (int t = threadIdx.x; t < (na + 2) * nc; t += blockDim.x) us[t] = make_double2(0.0, 0.0);
  double f2 = 0.0;
  for (int t = threadIdx.x; t < na * nb; t += blockDim.x) {
    double2 v = F[off + t];
    fs[t] = v;
    f2 += v.x * v.x + v.y * v.y;
  }
  auto block_sum = [&](double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
    __syncthreads();
    return s;
  };
  const double f2t = block_sum(f2);
  const double w = L.wc[m];
  const double* Ca = L.Ca + (size_t)m * na;
  const double* Cb = L.Cb + (size_t)m * nb;
  if (f2t > 0.0) {
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
      for (int colour = 0; colour < 2; ++colour) {
        for (int t = threadIdx.x; t < na * nb; t += blockDim.x) {
          const int i = t / nb, j = t - i * nb;
          if (((i + j) & 1) != colour) continue;
          const double R = L.Rr[i];
          const double c = Ca[i] + R * Cb[j];
          const int q = (i + 1) * nc + (j + 1);
          const double2 un = us[q + nc], uS = us[q - nc], ue = us[q + 1], uw = us[q - 1];
          const double a1 = L.ua[i], a2 = L.da[i], b1 = R * L.ub[j], b2 = R * L.db[j];
          const double2 fv = fs[t];
          const double tx = (fv.x - (a1 * un.x + a2 * uS.x + b1 * ue.x + b2 * uw.x)) / c;
          const double ty = (fv.y - (a1 * un.y + a2 * uS.y + b1 * ue.y + b2 * uw.y)) / c;
          const double2 old = us[q];
          us[q] = make_double2(old.x + w * (tx - old.x), old.y + w * (ty - old.y));
        }
        __syncthreads();
      }
      double r2 = 0.0;
      for (int t = threadIdx.x; t < na * nb; t += blockDim.x) {
        const int i = t / nb, j = t - i * nb;
        const double R = L.Rr[i];
        const double c = Ca[i] + R * Cb[j];
        const int q = (i + 1) * nc + (j + 1);
        const double2 un = us[q + nc], uS = us[q - nc], ue = us[q + 1], uw = us[q - 1], uc = us[q];
        const double a1 = L.ua[i], a2 = L.da[i], b1 = R * L.ub[j], b2 = R * L.db[j];
        const double2 fv = fs[t];
        const double rx = fv.x - (c * uc.x + a1 * un.x + a2 * uS.x + b1 * ue.x + b2 * uw.x);
        const double ry = fv.y - (c * uc.y + a1 * un.y + a2 * uS.y + b1 * ue.y + b2 * uw.y);
        r2 += rx * rx + ry * ry;
      }
      const double r2t = block_sum(r2);
      if (r2t <= rtol * rtol * f2t) break;
    }
  }
  for (int t = threadIdx.x; t < na * nb; t += blockDim.x) {
    const int i = t / nb, j = t - i * nb;
    U[off + t] = us[(i + 1) * nc + (j + 1)];
  }
}

// Volume-weighted squared defect: partial sums per (plane, block).
__global__ void __launch_bounds__(kThreads) k_norm_partial(LevelDev L, Batch bt, const double2* __restrict__ U,
                                                          const double2* __restrict__ F, double* __restrict__ partial) {
  // U == nullptr: norm of F itself (defect of the zero guess)
  __shared__ double red[kThreads / 64];
  const int p = blockIdx.y;
  const int slot = bt.slot[p], m = bt.mode[p];
  const size_t off = (size_t)slot * L.na * L.nb;
  const int cells = L.na * L.nb;
  double acc = 0.0;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < cells; t += gridDim.x * blockDim.x) {
    const int i = t / L.nb, j = t - i * L.nb;
    const double2 r = U ? resid_at(L, m, U + off, F + off, i, j) : F[off + t];
    acc += (r.x * r.x + r.y * r.y) * (L.va[i] * L.vb[j]);
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
    partial[(size_t)p * gridDim.x + blockIdx.x] = s;
  }
}

__global__ void k_norm_final(const double* __restrict__ partial, int nblk, int n, double* __restrict__ out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += partial[(size_t)p * nblk + b];
  out[p] = sqrt(s);
}

__global__ void k_fill_zero(double2* p, size_t n) {
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x)
    p[t] = make_double2(0.0, 0.0);
}

int grid_for(int cells) {
  int g = (cells + kThreads - 1) / kThreads;
  return g < 1 ? 1 : (g > 1024 ? 1024 : g);
}

constexpr size_t kSmoothLds = 48 * 1024;

}  // namespace

namespace smgk {

hipError_t mg_smooth_dir(const LevelDev& L, const Batch& b, double2* u, const double2* f, int n_sor, bool exact,
                         int dir, hipStream_t st) {
  if (b.n == 0) return hipSuccess;
  if (dir == 0) {
    // radial lines: tile of W columns spanning all rows
    const size_t row = sizeof(double2) * (L.na + 2) + (exact ? sizeof(double) * L.na / 2 : 0);
    int W = (int)((kSmoothLds - (exact ? 2 * sizeof(double) * L.na : 0)) / row) - 4;
    W = W < 2 ? 2 : (W > L.nb ? L.nb : W);
    if (W > 2 && (W & 1)) --W;
    const size_t lds = sizeof(double2) * (size_t)(L.na + 2) * (W + 4) +
                       (exact ? sizeof(double) * (size_t)(W / 2 + 2) * L.na : 0);
    if (exact)
      hipLaunchKernelGGL((k_smooth<0, true>), dim3((L.nb + W - 1) / W, b.n), dim3(kThreads), lds, st, L, b, u, f, n_sor, W);
    else
      hipLaunchKernelGGL((k_smooth<0, false>), dim3((L.nb + W - 1) / W, b.n), dim3(kThreads), lds, st, L, b, u, f, n_sor, W);
  } else {
    // polar lines: tile of T rows spanning all columns
    const size_t row = sizeof(double2) * (L.nb + 2) + (exact ? sizeof(double) * L.nb / 2 : 0);
    int T = (int)((kSmoothLds - (exact ? 2 * sizeof(double) * L.nb : 0)) / row) - 4;
    T = T < 2 ? 2 : (T > L.na ? L.na : T);
    if (T > 2 && (T & 1)) --T;
    const size_t lds = sizeof(double2) * (size_t)(T + 4) * (L.nb + 2) +
                       (exact ? sizeof(double) * (size_t)(T / 2 + 2) * L.nb : 0);
    if (exact)
      hipLaunchKernelGGL((k_smooth<1, true>), dim3((L.na + T - 1) / T, b.n), dim3(kThreads), lds, st, L, b, u, f, n_sor, T);
    else
      hipLaunchKernelGGL((k_smooth<1, false>), dim3((L.na + T - 1) / T, b.n), dim3(kThreads), lds, st, L, b, u, f, n_sor, T);
  }
  return hipGetLastError();
}

hipError_t mg_smooth(const LevelDev& L, const Batch& b, double2* u, const double2* f, int n_sor, bool exact,
                     hipStream_t st) {
  hipError_t e = mg_smooth_dir(L, b, u, f, n_sor, exact, 0, st);
  if (e != hipSuccess) return e;
  return mg_smooth_dir(L, b, u, f, n_sor, exact, 1, st);
}

hipError_t mg_residual(const LevelDev& L, const Batch& b, const double2* u, const double2* f, double2* r,
                       hipStream_t st) {
  if (b.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_residual, dim3(grid_for(L.na * L.nb), b.n), dim3(kThreads), 0, st, L, b, u, f, r);
  return hipGetLastError();
}

hipError_t mg_restrict_residual(const LevelDev& L, const LevelDev& C, const Batch& b, const double2* u,
                                const double2* f, double2* fc, double2* uc, hipStream_t st) {
  if (b.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_restrict, dim3(grid_for(C.na * C.nb), b.n), dim3(kThreads), 0, st, L, C, b, u, f, fc, uc);
  return hipGetLastError();
}

hipError_t mg_prolong_add(const LevelDev& L, const LevelDev& C, const Batch& b, double2* u, const double2* uc,
                          hipStream_t st) {
  if (b.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_prolong, dim3(grid_for(L.na * L.nb), b.n), dim3(kThreads), 0, st, L, C, b, u, uc);
  return hipGetLastError();
}

hipError_t mg_coarse_solve(const LevelDev& L, const Batch& b, double2* u, const double2* f, double rtol,
                           int max_sweeps, hipStream_t st) {
  if (b.n == 0) return hipSuccess;
  const size_t lds = sizeof(double2) * ((size_t)(L.na + 2) * (L.nb + 2) + (size_t)L.na * L.nb);
  hipLaunchKernelGGL(k_coarse, dim3(b.n), dim3(kThreads), lds, st, L, b, u, f, rtol, max_sweeps);
  return hipGetLastError();
}

hipError_t mg_norms(const LevelDev& L, const Batch& b, const double2* u, const double2* f, double* partial,
                    double* out, hipStream_t st) {
  if (b.n == 0) return hipSuccess;
  const int g = grid_for(L.na * L.nb) > 64 ? 64 : grid_for(L.na * L.nb);
  hipLaunchKernelGGL(k_norm_partial, dim3(g, b.n), dim3(kThreads), 0, st, L, b, u, f, partial);
  hipLaunchKernelGGL(k_norm_final, dim3((b.n + 255) / 256), dim3(256), 0, st, partial, g, b.n, out);
  return hipGetLastError();
}

hipError_t fill_zero(double2* p, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  size_t g = (n + kThreads - 1) / kThreads;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)g), dim3(kThreads), 0, st, p, n);
  return hipGetLastError();
}

}  // namespace smgk
