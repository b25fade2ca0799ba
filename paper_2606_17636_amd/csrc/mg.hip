// Per-mode geometric multigrid kernels (Sec. 3), batched over planes of one
// or several problems.  Block (x, y) works on list entry y (a plane of one
// problem) and tile x of it; the problem's level tables, arrays and launch
// shape come from its LvJob.  Entries beyond the device list length and
// tiles beyond the problem's own tile count return at once.
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
#include <algorithm>

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
__global__ void __launch_bounds__(kThreads) k_smooth(const LvJob* __restrict__ jobs, BatchRef bt, int n_sor) {
  using V = typename Vec<R>::T;
  extern __shared__ char smem[];
  V* sh = reinterpret_cast<V*>(smem);
  const int p = blockIdx.y;
  if (bt.count && p >= *bt.count) return;
  const int e = bt.ent[p];
  const LvJob& J = jobs[ent_prob(e)];
  if (!J.active || (int)blockIdx.x >= J.ntile[DIR]) return;
  const int slot = ent_slot(e);
  const int m = J.mode ? J.mode[slot] : slot;
  const LevelDev L = J.L;
  const int tile = J.tile[DIR], scratch_words = J.scratch[DIR], stage = J.stage[DIR];
  const int na = L.na, nb = L.nb;
  V* u = static_cast<V*>(J.u) + (size_t)slot * na * nb;
  const V* f = static_cast<const V*>(J.f) + (size_t)slot * na * nb;
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

// Common prologue of the per-cell kernels: resolve list entry blockIdx.y.
#define SMG_ENTRY(JOBS, BT)                                  \
  const int p = blockIdx.y;                                  \
  if ((BT).count && p >= *(BT).count) return;                \
  const int e = (BT).ent[p];                                 \
  const auto& J = (JOBS)[ent_prob(e)];                       \
  const int slot = ent_slot(e);                              \
  const int m = J.mode ? J.mode[slot] : slot;                \
  (void)m

__global__ void __launch_bounds__(kThreads) k_residual(const LvJob* __restrict__ jobs, BatchRef bt,
                                                      double2* __restrict__ Rout) {
  SMG_ENTRY(jobs, bt);
  const LevelDev L = J.L;
  const size_t off = (size_t)slot * L.na * L.nb;
  const double2* U = static_cast<const double2*>(J.u) + off;
  const double2* F = static_cast<const double2*>(J.f) + off;
  const int cells = L.na * L.nb;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < cells; t += gridDim.x * blockDim.x) {
    const int i = t / L.nb, j = t - i * L.nb;
    Rout[off + t] = resid_at<double>(L, m, U, F, i, j);
  }
}

// Coarse right-hand side = bilinear restriction of the fine residual; the
// coarse correction starts from zero.
template <typename R>
__global__ void __launch_bounds__(kThreads) k_restrict(const LvJob* __restrict__ jobs, BatchRef bt) {
  using V = typename Vec<R>::T;
  SMG_ENTRY(jobs, bt);
  if (!J.active) return;
  const LevelDev L = J.L, C = J.C;
  const size_t off = (size_t)slot * L.na * L.nb;
  const size_t offc = (size_t)slot * C.na * C.nb;
  const V* U = static_cast<const V*>(J.u) + off;
  const V* F = static_cast<const V*>(J.f) + off;
  V* FC = static_cast<V*>(J.fc) + offc;
  V* UC = static_cast<V*>(J.uc) + offc;
  const int cells = C.na * C.nb;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < cells; t += gridDim.x * blockDim.x) {
    const int I = t / C.nb, Jc = t - I * C.nb;
    V acc = mkv<R>(0, 0);
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const R wa = (R)L.rwa[2 * I + a];
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const R w = wa * (R)L.rwb[2 * Jc + b];
        const V r = resid_at<R>(L, m, U, F, 2 * I + a, 2 * Jc + b);
        acc = axpy<R>(w, r, acc);
      }
    }
    FC[t] = acc;
    UC[t] = mkv<R>(0, 0);
  }
}

template <typename R>
__global__ void __launch_bounds__(kThreads) k_prolong(const LvJob* __restrict__ jobs, BatchRef bt) {
  using V = typename Vec<R>::T;
  SMG_ENTRY(jobs, bt);
  if (!J.active) return;
  const LevelDev L = J.L, C = J.C;
  V* U = static_cast<V*>(J.u) + (size_t)slot * L.na * L.nb;
  const V* uc = static_cast<const V*>(J.uc) + (size_t)slot * C.na * C.nb;
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
    V ev = mkv<R>(0, 0);
    ev = axpy<R>(wa0 * wb0, uc[(size_t)a0 * C.nb + b0], ev);
    ev = axpy<R>(wa0 * wb1, uc[(size_t)a0 * C.nb + b1], ev);
    ev = axpy<R>(wa1 * wb0, uc[(size_t)a1 * C.nb + b0], ev);
    ev = axpy<R>(wa1 * wb1, uc[(size_t)a1 * C.nb + b1], ev);
    const V v = U[t];
    U[t] = mkv<R>(v.x + ev.x, v.y + ev.y);
  }
}

// Volume-weighted squared defect (FP64): partial sums per (list position,
// block).  use_u = 0: the defect of the zero guess (f itself).  With the
// mixed form the FP64 residual is also stored rounded to FP32 (the right-hand
// side of the next FP32 correction cycle) and the FP32 correction is zeroed.
__global__ void __launch_bounds__(kThreads) k_norm_partial(const NormJob* __restrict__ jobs, BatchRef bt, int use_u,
                                                          double* __restrict__ partial) {
  __shared__ double red[kThreads / 64];
  SMG_ENTRY(jobs, bt);
  const LevelDev L = J.L;
  const size_t off = (size_t)slot * L.na * L.nb;
  const double2* U = J.u + off;
  const double2* F = J.f + off;
  float2* R32 = J.r32 ? J.r32 + off : nullptr;
  float2* E32 = J.e32 ? J.e32 + off : nullptr;
  const int cells = L.na * L.nb;
  double acc = 0.0;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < cells; t += gridDim.x * blockDim.x) {
    const int i = t / L.nb, j = t - i * L.nb;
    const double2 r = use_u ? resid_at<double>(L, m, U, F, i, j) : F[t];
    if (R32) {
      R32[t] = make_float2((float)r.x, (float)r.y);
      E32[t] = make_float2(0.f, 0.f);
    }
    acc += (r.x * r.x + r.y * r.y) * (L.va[i] * L.vb[j]);
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double sum = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) sum += red[w];
    partial[(size_t)p * gridDim.x + blockIdx.x] = sum;
  }
}

// u (FP64) += e (FP32): the correction step of the mixed form.
__global__ void __launch_bounds__(kThreads) k_accumulate(const NormJob* __restrict__ jobs, BatchRef bt) {
  SMG_ENTRY(jobs, bt);
  const int cells = J.L.na * J.L.nb;
  const size_t off = (size_t)slot * cells;
  double2* U = J.u + off;
  const float2* E = J.e32 + off;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < cells; t += gridDim.x * blockDim.x) {
    const float2 ev = E[t];
    const double2 v = U[t];
    U[t] = make_double2(v.x + (double)ev.x, v.y + (double)ev.y);
  }
}

__global__ void k_fill_zero(double2* p, size_t n) {
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x)
    p[t] = make_double2(0.0, 0.0);
}

__global__ void k_copy(double2* __restrict__ d, const double2* __restrict__ s, size_t n) {
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) d[t] = s[t];
}

int grid_for(int cells) {
  int g = (cells + kThreads - 1) / kThreads;
  return g < 1 ? 1 : (g > 1024 ? 1024 : g);
}

constexpr size_t kSmoothLds = 60 * 1024;     // preferred per-block LDS
constexpr size_t kSmoothLdsMax = 64 * 1024;  // hard limit of a launch

}  // namespace

namespace smgk {

// Lines per tile so that a launch over `planes` planes has about
// target_blocks blocks, within the LDS budget; tables are staged in LDS when
// they fit.
bool smooth_shape(const LevelDev& L, int dir, bool exact, bool fp32, int target_blocks, int planes, SmoothShape* out) {
  const size_t vb = fp32 ? sizeof(float2) : sizeof(double2), rb = fp32 ? sizeof(float) : sizeof(double);
  const int npts = dir == 0 ? L.na : L.nb;    // points per line
  const int nlines = dir == 0 ? L.nb : L.na;  // lines in the plane
  auto bytes = [&](int t, bool stage) {
    const size_t nr = dir == 0 ? (size_t)L.na + 2 : (size_t)t + 4;
    const size_t nc = dir == 0 ? (size_t)t + 4 : (size_t)L.nb + 2;
    const size_t scratch = exact ? (size_t)(t / 2 + 2) * npts : 0;
    return vb * nr * nc + rb * (scratch + (stage ? 5 * nr + 4 * nc : 0));
  };
  if (planes < 1) planes = 1;
  const int want = (target_blocks + planes - 1) / planes;  // tiles per plane
  int tile = (nlines + want - 1) / want;
  if (tile < 2) tile = 2;
  if (tile > nlines) tile = nlines;
  while (tile > 2 && bytes(tile, true) > kSmoothLds) --tile;
  if (tile > 2 && (tile & 1)) --tile;
  const bool stage = bytes(tile, true) <= kSmoothLds;
  out->tile = tile;
  out->ntile = (nlines + tile - 1) / tile;
  out->stage = stage ? 1 : 0;
  out->scratch = exact ? (tile / 2 + 2) * npts : 0;
  out->lds = bytes(tile, stage);
  return out->lds <= kSmoothLdsMax;
}

template <typename R>
static hipError_t smooth_launch(const LvJob* jobs, const LvJob* hj, int n_prob, const BatchRef& b, int n_sor,
                                bool exact, int dir, hipStream_t st) {
  int gx = 0;
  size_t lds = 0;
  for (int q = 0; q < n_prob; ++q) {
    if (!hj[q].active) continue;
    const LevelDev& L = hj[q].L;
    const size_t vb = sizeof(typename Vec<R>::T), rb = sizeof(R);
    const int t = hj[q].tile[dir], npts = dir == 0 ? L.na : L.nb;
    const size_t nr = dir == 0 ? (size_t)L.na + 2 : (size_t)t + 4;
    const size_t nc = dir == 0 ? (size_t)t + 4 : (size_t)L.nb + 2;
    size_t bytes = vb * nr * nc + rb * ((size_t)hj[q].scratch[dir] + (hj[q].stage[dir] ? 5 * nr + 4 * nc : 0));
    (void)npts;
    if (bytes > lds) lds = bytes;
    if (hj[q].ntile[dir] > gx) gx = hj[q].ntile[dir];
  }
  if (gx == 0 || b.cap == 0) return hipSuccess;
  if (lds > kSmoothLdsMax) return hipErrorInvalidConfiguration;
  const dim3 grid(gx, b.cap);
  if (dir == 0) {
    if (exact) hipLaunchKernelGGL((k_smooth<0, true, R>), grid, dim3(kThreads), lds, st, jobs, b, n_sor);
    else hipLaunchKernelGGL((k_smooth<0, false, R>), grid, dim3(kThreads), lds, st, jobs, b, n_sor);
  } else {
    if (exact) hipLaunchKernelGGL((k_smooth<1, true, R>), grid, dim3(kThreads), lds, st, jobs, b, n_sor);
    else hipLaunchKernelGGL((k_smooth<1, false, R>), grid, dim3(kThreads), lds, st, jobs, b, n_sor);
  }
  return hipGetLastError();
}

hipError_t mg_smooth_dir(const LvJob* jobs, const LvJob* hj, int n_prob, const BatchRef& b, int n_sor, bool exact,
                         int dir, bool fp32, hipStream_t st) {
  return fp32 ? smooth_launch<float>(jobs, hj, n_prob, b, n_sor, exact, dir, st)
              : smooth_launch<double>(jobs, hj, n_prob, b, n_sor, exact, dir, st);
}

// blocks per plane of a per-cell launch: enough for the largest problem
static int cell_grid(const LvJob* hj, int n_prob, bool coarse, bool need_active) {
  int cells = 0;
  for (int q = 0; q < n_prob; ++q) {
    if (need_active && !hj[q].active) continue;
    const LevelDev& L = coarse ? hj[q].C : hj[q].L;
    cells = std::max(cells, L.na * L.nb);
  }
  return cells ? grid_for(cells) : 0;
}

hipError_t mg_residual(const LvJob* jobs, const LvJob* hj, int n_prob, const BatchRef& b, double2* r, hipStream_t st) {
  const int g = cell_grid(hj, n_prob, false, false);
  if (!g || !b.cap) return hipSuccess;
  hipLaunchKernelGGL(k_residual, dim3(g, b.cap), dim3(kThreads), 0, st, jobs, b, r);
  return hipGetLastError();
}

hipError_t mg_restrict(const LvJob* jobs, const LvJob* hj, int n_prob, const BatchRef& b, bool fp32, hipStream_t st) {
  const int g = cell_grid(hj, n_prob, true, true);
  if (!g || !b.cap) return hipSuccess;
  if (fp32) hipLaunchKernelGGL(k_restrict<float>, dim3(g, b.cap), dim3(kThreads), 0, st, jobs, b);
  else hipLaunchKernelGGL(k_restrict<double>, dim3(g, b.cap), dim3(kThreads), 0, st, jobs, b);
  return hipGetLastError();
}

hipError_t mg_prolong(const LvJob* jobs, const LvJob* hj, int n_prob, const BatchRef& b, bool fp32, hipStream_t st) {
  const int g = cell_grid(hj, n_prob, false, true);
  if (!g || !b.cap) return hipSuccess;
  if (fp32) hipLaunchKernelGGL(k_prolong<float>, dim3(g, b.cap), dim3(kThreads), 0, st, jobs, b);
  else hipLaunchKernelGGL(k_prolong<double>, dim3(g, b.cap), dim3(kThreads), 0, st, jobs, b);
  return hipGetLastError();
}

int norm_blocks(const NormJob* hj, int n_prob) {
  int cells = 0;
  for (int q = 0; q < n_prob; ++q) cells = std::max(cells, hj[q].L.na * hj[q].L.nb);
  const int g = grid_for(cells);
  return g > 64 ? 64 : g;
}

hipError_t mg_norm_partial(const NormJob* jobs, const NormJob* hj, int n_prob, const BatchRef& b, bool use_u,
                           double* partial, int nblk, hipStream_t st) {
  (void)hj; (void)n_prob;
  if (!b.cap) return hipSuccess;
  hipLaunchKernelGGL(k_norm_partial, dim3(nblk, b.cap), dim3(kThreads), 0, st, jobs, b, use_u ? 1 : 0, partial);
  return hipGetLastError();
}

hipError_t mg_accumulate(const NormJob* jobs, const NormJob* hj, int n_prob, const BatchRef& b, hipStream_t st) {
  int cells = 0;
  for (int q = 0; q < n_prob; ++q) cells = std::max(cells, hj[q].L.na * hj[q].L.nb);
  if (!cells || !b.cap) return hipSuccess;
  hipLaunchKernelGGL(k_accumulate, dim3(grid_for(cells), b.cap), dim3(kThreads), 0, st, jobs, b);
  return hipGetLastError();
}

hipError_t fill_zero(double2* p, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  size_t g = (n + kThreads - 1) / kThreads;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)g), dim3(kThreads), 0, st, p, n);
  return hipGetLastError();
}

hipError_t copy_planes(double2* dst, const double2* src, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  size_t g = (n + kThreads - 1) / kThreads;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)g), dim3(kThreads), 0, st, dst, src, n);
  return hipGetLastError();
}

}  // namespace smgk
