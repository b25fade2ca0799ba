// Per-mode geometric multigrid kernels (Sec. 3), batched over planes.
//
// A level stores each plane as an interleaved complex array [na][nb] (b
// fastest), FP64 (double2) or, for the smoothing and transfers of the mixed
// precision form, FP32 (float2); the kernels are templates on the real type
// R.  The stencil tables are FP64 in memory and are rounded to R when
// staged.  The operator of mode m at (i, j) is
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
// even-odd SOR passes of every line run as point updates in LDS, or (exact
// variant) each line is solved by the Thomas algorithm.
#include "smg_internal.h"
#include "vec.h"

namespace {

constexpr int kThreads = 256;

// Residual f - L u at (i, j) of one plane, reading u from global memory (R).
template <typename R>
__device__ __forceinline__ typename Vec<R>::T resid_at(const LevelDev& L, int m, const typename Vec<R>::T* __restrict__ u,
                                                       const typename Vec<R>::T* __restrict__ f, int i, int j) {
  using V = typename Vec<R>::T;
  const int na = L.na, nb = L.nb;
  const size_t row = (size_t)i * nb;
  const int ip = min(i + 1, na - 1), im = max(i - 1, 0);
  const int jp = min(j + 1, nb - 1), jm = max(j - 1, 0);
  const R Rr = (R)L.Rr[i];
  const R c = (R)L.Ca[(size_t)m * na + i] + Rr * (R)L.Cb[(size_t)m * nb + j];
  const V uc = u[row + j];
  V acc = mkv<R>(c * uc.x, c * uc.y);
  acc = axpy<R>((R)L.ua[i], u[(size_t)ip * nb + j], acc);
  acc = axpy<R>((R)L.da[i], u[(size_t)im * nb + j], acc);
  acc = axpy<R>(Rr * (R)L.ub[j], u[row + jp], acc);
  acc = axpy<R>(Rr * (R)L.db[j], u[row + jm], acc);
  const V fv = f[row + j];
  return mkv<R>(fv.x - acc.x, fv.y - acc.y);
}

// ---------------------------------------------------------------------------
// Smoother.  DIR = 1: polar lines (rows i, points along j); tile = rows
// [i0-2, i0+T+2) x all columns.  DIR = 0: radial lines (columns j, points
// along i); tile = all rows x columns [j0-2, j0+W+2).  LDS holds the tile
// with one zero column/row of padding at the ends of the lines.
// ---------------------------------------------------------------------------
template <int DIR, bool EXACT, typename R>
__global__ void __launch_bounds__(kThreads) k_smooth(LevelDev L, Batch bt, typename Vec<R>::T* __restrict__ U,
                                                    const typename Vec<R>::T* __restrict__ F, int n_sor, int tile,
                                                    int scratch_words, int stage) {
  using V = typename Vec<R>::T;
  extern __shared__ char smem[];
  V* sh = reinterpret_cast<V*>(smem);
  const int p = blockIdx.y;
  const int slot = bt.slot[p], m = bt.mode[p];
  const int na = L.na, nb = L.nb;
  V* u = U + (size_t)slot * na * nb;
  const V* f = F + (size_t)slot * na * nb;
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
    V v = mkv<R>(0, 0);
    if (i >= 0 && i < na && j >= 0 && j < nb) v = u[(size_t)i * nb + j];
    sh[t] = v;
  }
  // line range of this tile (the coordinate across the lines)
  const int lbeg = blockIdx.x * tile;                     // first owned line
  const int lend = min(lbeg + tile, DIR == 1 ? na : nb);  // one past the last owned line
  const int nlines_total = DIR == 1 ? na : nb;
  const int npts = DIR == 1 ? nb : na;                    // points per line
  // scratch for the exact line solve: one row of Thomas factors per line
  R* cp = reinterpret_cast<R*>(sh + nr * nc);
  // the 1D stencil tables of this tile and mode (per row ua, da, R, Ca,
  // omega of the polar line; per column ub, db, Cb, omega of the radial
  // line), staged in LDS (rounded to R); indexed by the tile-local row
  // rr = i - r0 and column cc = j - c0.
  R* t0 = cp + scratch_words;
  R *t1 = t0 + nr, *t2 = t1 + nr, *t3 = t2 + nr, *t4 = t3 + nr;
  R *c1 = t4 + nr, *c2 = c1 + nc, *c3 = c2 + nc, *c4 = c3 + nc;
  if (stage) {
    for (int rr = threadIdx.x; rr < nr; rr += blockDim.x) {
      const int i = r0 + rr;
      const bool in = i >= 0 && i < na;
      t0[rr] = in ? (R)L.ua[i] : (R)0;
      t1[rr] = in ? (R)L.da[i] : (R)0;
      t2[rr] = in ? (R)L.Rr[i] : (R)0;
      t3[rr] = in ? (R)L.Ca[(size_t)m * na + i] : (R)1;
      t4[rr] = in ? (R)L.wb[(size_t)m * na + i] : (R)0;
    }
    for (int cc = threadIdx.x; cc < nc; cc += blockDim.x) {
      const int j = c0 + cc;
      const bool in = j >= 0 && j < nb;
      c1[cc] = in ? (R)L.ub[j] : (R)0;
      c2[cc] = in ? (R)L.db[j] : (R)0;
      c3[cc] = in ? (R)L.Cb[(size_t)m * nb + j] : (R)0;
      c4[cc] = in ? (R)L.wr[(size_t)m * nb + j] : (R)0;
    }
  }
  __syncthreads();
  // table access: staged copy or the FP64 tables in place (rows and
  // columns outside the plane are never read)
  auto tU = [&](int rr) { return stage ? t0[rr] : (R)L.ua[r0 + rr]; };
  auto tD = [&](int rr) { return stage ? t1[rr] : (R)L.da[r0 + rr]; };
  auto tR = [&](int rr) { return stage ? t2[rr] : (R)L.Rr[r0 + rr]; };
  auto tC = [&](int rr) { return stage ? t3[rr] : (R)L.Ca[(size_t)m * na + r0 + rr]; };
  auto tW = [&](int rr) { return stage ? t4[rr] : (R)L.wb[(size_t)m * na + r0 + rr]; };
  auto cU = [&](int cc) { return stage ? c1[cc] : (R)L.ub[c0 + cc]; };
  auto cD = [&](int cc) { return stage ? c2[cc] : (R)L.db[c0 + cc]; };
  auto cC = [&](int cc) { return stage ? c3[cc] : (R)L.Cb[(size_t)m * nb + c0 + cc]; };
  auto cW = [&](int cc) { return stage ? c4[cc] : (R)L.wr[(size_t)m * nb + c0 + cc]; };
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
        R* cpl = cp + t * npts;
        V prev = mkv<R>(0, 0);
        R cprev = 0;
        for (int k = 0; k < npts; ++k) {
          const int i = DIR == 1 ? line : k;
          const int j = DIR == 1 ? k : line;
          const int rr = i - r0, cc = j - c0;
          const R Rr = tR(rr);
          const R c = tC(rr) + Rr * cC(cc);
          R lo, up, w1, w2;
          V o1, o2;
          if (DIR == 1) {  // line along j; fixed neighbours i+1, i-1
            lo = Rr * cD(cc); up = Rr * cU(cc);
            o1 = sh[(rr + 1) * nc + cc]; o2 = sh[(rr - 1) * nc + cc];
            w1 = tU(rr); w2 = tD(rr);
          } else {         // line along i; fixed neighbours j+1, j-1
            lo = tD(rr); up = tU(rr);
            o1 = sh[rr * nc + cc + 1]; o2 = sh[rr * nc + cc - 1];
            w1 = Rr * cU(cc); w2 = Rr * cD(cc);
          }
          const V fv = f[(size_t)i * nb + j];
          const R rx = fv.x - (w1 * o1.x + w2 * o2.x);
          const R ry = fv.y - (w1 * o1.y + w2 * o2.y);
          const R den = c - lo * cprev;
          cprev = up / den;
          cpl[k] = cprev;
          prev = mkv<R>((rx - lo * prev.x) / den, (ry - lo * prev.y) / den);
          sh[rr * nc + cc] = prev;
        }
        for (int k = npts - 2; k >= 0; --k) {
          const int i = DIR == 1 ? line : k;
          const int j = DIR == 1 ? k : line;
          const int rr = i - r0, cc = j - c0;
          const V nx = DIR == 1 ? sh[rr * nc + cc + 1] : sh[(rr + 1) * nc + cc];
          const V d = sh[rr * nc + cc];
          sh[rr * nc + cc] = mkv<R>(d.x - cpl[k] * nx.x, d.y - cpl[k] * nx.y);
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
          V* me = &sh[rr * nc + cc];
          const V un = sh[(rr + 1) * nc + cc];
          const V us = sh[(rr - 1) * nc + cc];
          const V ue = sh[rr * nc + cc + 1];
          const V uw = sh[rr * nc + cc - 1];
          const R Rr = tR(rr);
          const R c = tC(rr) + Rr * cC(cc);
          const R w = DIR == 1 ? tW(rr) : cW(cc);
          const R ua = tU(rr), da = tD(rr), ub = Rr * cU(cc), db = Rr * cD(cc);
          const V fv = f[(size_t)i * nb + j];
          const R sx = ua * un.x + da * us.x + ub * ue.x + db * uw.x;
          const R sy = ua * un.y + da * us.y + ub * ue.y + db * uw.y;
          const V old = *me;
          const R tx = (fv.x - sx) / c, ty = (fv.y - sy) / c;
          *me = mkv<R>(old.x + w * (tx - old.x), old.y + w * (ty - old.y));
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
    Rout[off + t] = resid_at<double>(L, m, U + off, F + off, i, j);
  }
}

// Coarse right-hand side = bilinear restriction of the fine residual; the
// coarse correction starts from zero.
template <typename R>
__global__ void __launch_bounds__(kThreads) k_restrict(LevelDev L, LevelDev C, Batch bt,
                                                      const typename Vec<R>::T* __restrict__ U,
                                                      const typename Vec<R>::T* __restrict__ F,
                                                      typename Vec<R>::T* __restrict__ FC,
                                                      typename Vec<R>::T* __restrict__ UC) {
  using V = typename Vec<R>::T;
  const int p = blockIdx.y;
  const int slot = bt.slot[p], m = bt.mode[p];
  const size_t off = (size_t)slot * L.na * L.nb;
  const size_t offc = (size_t)slot * C.na * C.nb;
  const int cells = C.na * C.nb;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < cells; t += gridDim.x * blockDim.x) {
    const int I = t / C.nb, J = t - I * C.nb;
    V acc = mkv<R>(0, 0);
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const R wa = (R)L.rwa[2 * I + a];
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const R w = wa * (R)L.rwb[2 * J + b];
        const V r = resid_at<R>(L, m, U + off, F + off, 2 * I + a, 2 * J + b);
        acc = axpy<R>(w, r, acc);
      }
    }
    FC[offc + t] = acc;
    UC[offc + t] = mkv<R>(0, 0);
  }
}

template <typename R>
__global__ void __launch_bounds__(kThreads) k_prolong(LevelDev L, LevelDev C, Batch bt, typename Vec<R>::T* __restrict__ U,
                                                     const typename Vec<R>::T* __restrict__ UC) {
  using V = typename Vec<R>::T;
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
    const R wa0 = (R)L.pa_w0[i], wa1 = (R)L.pa_w1[i];
    const R wb0 = (R)pbw0[j], wb1 = (R)pbw1[j];
    const V* uc = UC + offc;
    V e = mkv<R>(0, 0);
    e = axpy<R>(wa0 * wb0, uc[(size_t)a0 * C.nb + b0], e);
    e = axpy<R>(wa0 * wb1, uc[(size_t)a0 * C.nb + b1], e);
    e = axpy<R>(wa1 * wb0, uc[(size_t)a1 * C.nb + b0], e);
    e = axpy<R>(wa1 * wb1, uc[(size_t)a1 * C.nb + b1], e);
    const V v = U[off + t];
    U[off + t] = mkv<R>(v.x + e.x, v.y + e.y);
  }
}

// Volume-weighted squared defect (FP64): partial sums per (plane, block).
// U == nullptr: norm of F itself (defect of the zero guess).  When R32 is
// non-null the FP64 residual is also stored rounded to FP32 (the right-hand
// side of the next FP32 correction cycle of the mixed form) and the FP32
// correction E32 is reset to zero.
__global__ void __launch_bounds__(kThreads) k_norm_partial(LevelDev L, Batch bt, const double2* __restrict__ U,
                                                          const double2* __restrict__ F, double* __restrict__ partial,
                                                          float2* __restrict__ R32, float2* __restrict__ E32) {
  __shared__ double red[kThreads / 64];
  const int p = blockIdx.y;
  const int slot = bt.slot[p], m = bt.mode[p];
  const size_t off = (size_t)slot * L.na * L.nb;
  const int cells = L.na * L.nb;
  double acc = 0.0;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < cells; t += gridDim.x * blockDim.x) {
    const int i = t / L.nb, j = t - i * L.nb;
    const double2 r = U ? resid_at<double>(L, m, U + off, F + off, i, j) : F[off + t];
    if (R32) {
      R32[off + t] = make_float2((float)r.x, (float)r.y);
      E32[off + t] = make_float2(0.f, 0.f);
    }
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

// u (FP64) += e (FP32): the correction step of the mixed form.
__global__ void __launch_bounds__(kThreads) k_accumulate(int cells, Batch bt, double2* __restrict__ U,
                                                        const float2* __restrict__ E) {
  const int p = blockIdx.y;
  const size_t off = (size_t)bt.slot[p] * cells;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < cells; t += gridDim.x * blockDim.x) {
    const float2 e = E[off + t];
    const double2 v = U[off + t];
    U[off + t] = make_double2(v.x + (double)e.x, v.y + (double)e.y);
  }
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

template <typename R>
hipError_t smooth_dir(const LevelDev& L, const Batch& b, typename Vec<R>::T* u, const typename Vec<R>::T* f, int n_sor,
                      bool exact, int dir, hipStream_t st) {
  using V = typename Vec<R>::T;
  if (b.n == 0) return hipSuccess;
  // LDS per block: tile (lines + 4 halo) x (points + 2), Thomas scratch for
  // the exact variant, and the staged 1D tables (5 per row, 4 per column).
  const int npts = dir == 0 ? L.na : L.nb;       // points per line
  const int nlines = dir == 0 ? L.nb : L.na;     // lines in the plane
  auto bytes = [&](int t, bool stage) {
    const size_t nr = dir == 0 ? (size_t)L.na + 2 : (size_t)t + 4;
    const size_t nc = dir == 0 ? (size_t)t + 4 : (size_t)L.nb + 2;
    const size_t scratch = exact ? (size_t)(t / 2 + 2) * npts : 0;
    return sizeof(V) * nr * nc + sizeof(R) * (scratch + (stage ? 5 * nr + 4 * nc : 0));
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
      hipLaunchKernelGGL((k_smooth<0, true, R>), grid, dim3(kThreads), lds, st, L, b, u, f, n_sor, tile, scratch, sg);
    else
      hipLaunchKernelGGL((k_smooth<0, false, R>), grid, dim3(kThreads), lds, st, L, b, u, f, n_sor, tile, scratch, sg);
  } else {
    if (exact)
      hipLaunchKernelGGL((k_smooth<1, true, R>), grid, dim3(kThreads), lds, st, L, b, u, f, n_sor, tile, scratch, sg);
    else
      hipLaunchKernelGGL((k_smooth<1, false, R>), grid, dim3(kThreads), lds, st, L, b, u, f, n_sor, tile, scratch, sg);
  }
  return hipGetLastError();
}

}  // namespace

namespace smgk {

hipError_t mg_smooth_dir(const LevelDev& L, const Batch& b, double2* u, const double2* f, int n_sor, bool exact,
                         int dir, hipStream_t st) {
  return smooth_dir<double>(L, b, u, f, n_sor, exact, dir, st);
}

hipError_t mg_smooth_dir32(const LevelDev& L, const Batch& b, float2* u, const float2* f, int n_sor, bool exact,
                           int dir, hipStream_t st) {
  return smooth_dir<float>(L, b, u, f, n_sor, exact, dir, st);
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
  hipLaunchKernelGGL(k_restrict<double>, dim3(grid_for(C.na * C.nb), b.n), dim3(kThreads), 0, st, L, C, b, u, f, fc, uc);
  return hipGetLastError();
}

hipError_t mg_restrict_residual32(const LevelDev& L, const LevelDev& C, const Batch& b, const float2* u,
                                  const float2* f, float2* fc, float2* uc, hipStream_t st) {
  if (b.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_restrict<float>, dim3(grid_for(C.na * C.nb), b.n), dim3(kThreads), 0, st, L, C, b, u, f, fc, uc);
  return hipGetLastError();
}

hipError_t mg_prolong_add(const LevelDev& L, const LevelDev& C, const Batch& b, double2* u, const double2* uc,
                          hipStream_t st) {
  if (b.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_prolong<double>, dim3(grid_for(L.na * L.nb), b.n), dim3(kThreads), 0, st, L, C, b, u, uc);
  return hipGetLastError();
}

hipError_t mg_prolong_add32(const LevelDev& L, const LevelDev& C, const Batch& b, float2* u, const float2* uc,
                            hipStream_t st) {
  if (b.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_prolong<float>, dim3(grid_for(L.na * L.nb), b.n), dim3(kThreads), 0, st, L, C, b, u, uc);
  return hipGetLastError();
}

hipError_t mg_norms(const LevelDev& L, const Batch& b, const double2* u, const double2* f, double* partial,
                    double* out, hipStream_t st, float2* r32, float2* e32) {
  if (b.n == 0) return hipSuccess;
  const int g = grid_for(L.na * L.nb) > 64 ? 64 : grid_for(L.na * L.nb);
  hipLaunchKernelGGL(k_norm_partial, dim3(g, b.n), dim3(kThreads), 0, st, L, b, u, f, partial, r32, e32);
  hipLaunchKernelGGL(k_norm_final, dim3((b.n + 255) / 256), dim3(256), 0, st, partial, g, b.n, out);
  return hipGetLastError();
}

hipError_t mg_accumulate(const LevelDev& L, const Batch& b, double2* u, const float2* e, hipStream_t st) {
  if (b.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_accumulate, dim3(grid_for(L.na * L.nb), b.n), dim3(kThreads), 0, st, L.na * L.nb, b, u, e);
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
