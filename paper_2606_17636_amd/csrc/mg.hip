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
                                                    const double2* __restrict__ F, int n_sor, int tile,
                                                    int scratch_doubles, int stage) {
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
  // the 1D stencil tables of this tile and mode (per row ua, da, R, Ca,
  // omega of the polar line; per column ub, db, Cb, omega of the radial
  // line), staged in LDS when they fit, else read in place; indexed by the
  // tile-local row rr = i - r0 and column cc = j - c0.
  const double *trU, *trD, *trR, *trC, *trW, *tcU, *tcD, *tcC, *tcW;
  if (stage) {
    double* t0 = cp + scratch_doubles;
    double* t1 = t0 + nr;
    double* t2 = t1 + nr;
    double* t3 = t2 + nr;
    double* t4 = t3 + nr;
    double* c1 = t4 + nr;
    double* c2 = c1 + nc;
    double* c3 = c2 + nc;
    double* c4 = c3 + nc;
    for (int rr = threadIdx.x; rr < nr; rr += blockDim.x) {
      const int i = r0 + rr;
      const bool in = i >= 0 && i < na;
      t0[rr] = in ? L.ua[i] : 0.0;
      t1[rr] = in ? L.da[i] : 0.0;
      t2[rr] = in ? L.Rr[i] : 0.0;
      t3[rr] = in ? L.Ca[(size_t)m * na + i] : 1.0;
      t4[rr] = in ? L.wb[(size_t)m * na + i] : 0.0;
    }
    for (int cc = threadIdx.x; cc < nc; cc += blockDim.x) {
      const int j = c0 + cc;
      const bool in = j >= 0 && j < nb;
      c1[cc] = in ? L.ub[j] : 0.0;
      c2[cc] = in ? L.db[j] : 0.0;
      c3[cc] = in ? L.Cb[(size_t)m * nb + j] : 0.0;
      c4[cc] = in ? L.wr[(size_t)m * nb + j] : 0.0;
    }
    trU = t0; trD = t1; trR = t2; trC = t3; trW = t4;
    tcU = c1; tcD = c2; tcC = c3; tcW = c4;
    __syncthreads();
  } else {
    // rows and columns outside the plane are never read
    trU = L.ua + r0; trD = L.da + r0; trR = L.Rr + r0;
    trC = L.Ca + (size_t)m * na + r0; trW = L.wb + (size_t)m * na + r0;
    tcU = L.ub + c0; tcD = L.db + c0; tcC = L.Cb + (size_t)m * nb + c0; tcW = L.wr + (size_t)m * nb + c0;
  }
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
          const double R = trR[rr];
          const double c = trC[rr] + R * tcC[cc];
          double lo, up;
          double2 o1, o2;
          double w1, w2;
          if (DIR == 1) {  // line along j; fixed neighbours i+1, i-1
            lo = R * tcD[cc]; up = R * tcU[cc];
            o1 = sh[(rr + 1) * nc + cc]; o2 = sh[(rr - 1) * nc + cc];
            w1 = trU[rr]; w2 = trD[rr];
          } else {         // line along i; fixed neighbours j+1, j-1
            lo = trD[rr]; up = trU[rr];
            o1 = sh[rr * nc + cc + 1]; o2 = sh[rr * nc + cc - 1];
            w1 = R * tcU[cc]; w2 = R * tcD[cc];
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
          const double R = trR[rr];
          const double c = trC[rr] + R * tcC[cc];
          const double w = DIR == 1 ? trW[rr] : tcW[cc];
          const double ua = trU[rr], da = trD[rr], ub = R * tcU[cc], db = R * tcD[cc];
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

constexpr size_t kSmoothLds = 60 * 1024;     // preferred per-block LDS
constexpr size_t kSmoothLdsMax = 64 * 1024;  // hard limit of a launch

// Lines per tile so that a launch over n_planes planes has about two blocks
// per compute unit (512 blocks) when the planes allow it.
int par_tile(int n_lines, int n_planes) {
  const int want = (512 + n_planes - 1) / n_planes;  // tiles per plane
  int t = (n_lines + want - 1) / want;
  return t < 2 ? 2 : t;
}

}  // namespace

namespace smgk {

hipError_t mg_smooth_dir(const LevelDev& L, const Batch& b, double2* u, const double2* f, int n_sor, bool exact,
                         int dir, hipStream_t st) {
  if (b.n == 0) return hipSuccess;
  // LDS per block: tile (lines + 4 halo) x (points + 2), Thomas scratch for
  // the exact variant, and the staged 1D tables (5 per row, 4 per column).
  const int npts = dir == 0 ? L.na : L.nb;       // points per line
  const int nlines = dir == 0 ? L.nb : L.na;     // lines in the plane
  auto bytes = [&](int t, bool stage) {
    const size_t nr = dir == 0 ? (size_t)L.na + 2 : (size_t)t + 4;
    const size_t nc = dir == 0 ? (size_t)t + 4 : (size_t)L.nb + 2;
    const size_t scratch = exact ? (size_t)(t / 2 + 2) * npts : 0;
    return sizeof(double2) * nr * nc + sizeof(double) * (scratch + (stage ? 5 * nr + 4 * nc : 0));
  };
  int tile = par_tile(nlines, b.n);
  if (tile > nlines) tile = nlines;
  while (tile > 2 && bytes(tile, true) > kSmoothLds) --tile;
  if (tile > 2 && (tile & 1)) --tile;
  const bool stage = bytes(tile, true) <= kSmoothLds;
  const size_t lds = bytes(tile, stage);
  if (lds > kSmoothLdsMax) return hipErrorInvalidConfiguration;
  const int scratch = exact ? (tile / 2 + 2) * npts : 0;
  const dim3 grid((nlines + tile - 1) / tile, b.n);
  const int sg = stage ? 1 : 0;
  if (dir == 0) {
    if (exact)
      hipLaunchKernelGGL((k_smooth<0, true>), grid, dim3(kThreads), lds, st, L, b, u, f, n_sor, tile, scratch, sg);
    else
      hipLaunchKernelGGL((k_smooth<0, false>), grid, dim3(kThreads), lds, st, L, b, u, f, n_sor, tile, scratch, sg);
  } else {
    if (exact)
      hipLaunchKernelGGL((k_smooth<1, true>), grid, dim3(kThreads), lds, st, L, b, u, f, n_sor, tile, scratch, sg);
    else
      hipLaunchKernelGGL((k_smooth<1, false>), grid, dim3(kThreads), lds, st, L, b, u, f, n_sor, tile, scratch, sg);
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
