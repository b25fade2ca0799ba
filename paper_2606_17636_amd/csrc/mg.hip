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
// even-odd SOR passes of every line run in registers (relax_dev.h), or
// (exact variant) each line is solved by the Thomas algorithm.  Each level
// has two iterate arrays: radial-line launches read u and write u2,
// polar-line launches read u2 and write u, so no block of a launch reads
// lines another block of it writes.  Blocks are renumbered so that the tiles
// of a plane run on one XCD and share its L2.
#include <algorithm>
#include <type_traits>

#include <hip/hip_ext.h>

#include "batch_dev.h"
#include "relax_dev.h"
#include "smg_internal.h"
#include "vec.h"

namespace {

constexpr int kThreads = 256;
constexpr unsigned kXcds = 8;  // accelerator complex dies of the device, each with its own L2

// Residual f - L u at (i, j) of one plane, reading u from global memory (R).
template <typename R>
__device__ __forceinline__ typename Vec<R>::T resid_at(const LevelDev& L, int m, const typename Vec<R>::T* __restrict__ u,
                                                       const typename Vec<R>::T* __restrict__ f, int i, int j) {
  using V = typename Vec<R>::T;
  const int na = L.na, nb = L.nb;
  const auto ug = gbl(u);
  const size_t row = (size_t)i * nb;
  const int ip = min(i + 1, na - 1), im = max(i - 1, 0);
  const int jp = min(j + 1, nb - 1), jm = max(j - 1, 0);
  const R Rr = (R)gbl(L.Rr)[i];
  const R c = (R)gbl(L.Ca)[(size_t)m * na + i] + Rr * (R)gbl(L.Cb)[(size_t)m * nb + j];
  const V uc = ug[row + j];
  V acc = mkv<R>(c * uc.x, c * uc.y);
  acc = axpy<R>((R)gbl(L.ua)[i], ug[(size_t)ip * nb + j], acc);
  acc = axpy<R>((R)gbl(L.da)[i], ug[(size_t)im * nb + j], acc);
  acc = axpy<R>(Rr * (R)gbl(L.ub)[j], ug[row + jp], acc);
  acc = axpy<R>(Rr * (R)gbl(L.db)[j], ug[row + jm], acc);
  const V fv = gbl(f)[row + j];
  return mkv<R>(fv.x - acc.x, fv.y - acc.y);
}

// Bilinear interpolation of the coarse correction uc (one plane, C.nb
// columns) at fine cell (i, j); the b-direction weights depend on the parity
// of the mode (par).
template <typename R, typename P>
__device__ __forceinline__ typename Vec<R>::T coarse_corr(const LevelDev& L, int cnb, P uc, int par, int i, int j) {
  using V = typename Vec<R>::T;
  const int a0 = gbl(L.pa_i0)[i], a1 = gbl(L.pa_i1)[i];
  const int b0 = gbl(L.pb_i0)[par * L.nb + j], b1 = gbl(L.pb_i1)[par * L.nb + j];
  const R wa0 = (R)gbl(L.pa_w0)[i], wa1 = (R)gbl(L.pa_w1)[i];
  const R wb0 = (R)gbl(L.pb_w0)[par * L.nb + j], wb1 = (R)gbl(L.pb_w1)[par * L.nb + j];
  V ev = mkv<R>(0, 0);
  ev = axpy<R>(wa0 * wb0, (V)uc[(size_t)a0 * cnb + b0], ev);
  ev = axpy<R>(wa0 * wb1, (V)uc[(size_t)a0 * cnb + b1], ev);
  ev = axpy<R>(wa1 * wb0, (V)uc[(size_t)a1 * cnb + b0], ev);
  ev = axpy<R>(wa1 * wb1, (V)uc[(size_t)a1 * cnb + b1], ev);
  return ev;
}

// ---------------------------------------------------------------------------
// Smoother.  DIR = 1: polar lines (rows i, points along j); tile = rows
// [i0-2, i0+T+2) x all columns.  DIR = 0: radial lines (columns j, points
// along i); tile = all rows x columns [j0-2, j0+W+2).  LDS holds the u tile
// with one zero column/row of padding at the ends of the lines, f of the
// lines the block relaxes (owned lines and the inner halo line on each side)
// in the same layout, and the 1D stencil tables of the tile rounded to R.
// The first batch of global reads is issued before any LDS store; the
// colours then run out of LDS and registers.  With PROLONG the launch first applies
// the coarse-grid correction: every u value entering the tile (halo lines
// included) gets the interpolated coarse correction added, so the owned
// lines written back carry it and no separate prolongation pass is needed.
// With ACC (polar lines, FP32 correction of the mixed form) the owned lines
// are added to the FP64 iterate instead of being stored, which is the
// correction step of the mixed form done by the V-cycle's last launch.
// With ZERO (radial lines) the launch takes u = 0 without reading it.
// ---------------------------------------------------------------------------
// LDS bytes of a smoother block: u tile, f tile (the SOR variant; the exact
// variant reads each f value once, from global memory), exact-line scratch
// and tables.  A launch that applies the coarse correction (prolong) also
// holds the prolongation indices and weights of the tile's rows and columns.
template <typename R>
__host__ __device__ inline size_t smooth_lds_bytes(int dir, int na, int nb, int tile, bool exact, int scratch,
                                                   bool prolong = false) {
  const size_t nr = dir == 0 ? (size_t)na + 2 : (size_t)tile + 4;
  const size_t nc = dir == 0 ? (size_t)odd_stride(tile + 4) : (size_t)nb + 2;
  return (exact ? 1 : 2) * sizeof(typename Vec<R>::T) * nr * nc + sizeof(R) * ((size_t)scratch + 5 * nr + 4 * nc) +
         (prolong ? (nr + nc) * (2 * sizeof(int) + 2 * sizeof(R)) : 0);
}

// How a launch obtains u: from the level array, from the level array plus
// the prolonged coarse correction, or as zero (the mixed form's correction
// cycle starts from e = 0, so its first launch reads nothing).
constexpr int kInLoad = 0, kInProlong = 1, kInZero = 2;

template <int DIR, bool EXACT, int PMAX, typename R, int NT, int IN, bool ACC = false>
__global__ void __launch_bounds__(NT) k_smooth(const LvJob* __restrict__ jobs, BatchRef bt, int n_sor) {
  constexpr bool PROLONG = IN == kInProlong, ZERO = IN == kInZero;
  using V = typename Vec<R>::T;
  extern __shared__ char smem[];
  V* sh = reinterpret_cast<V*>(smem);
  // XCD-aware block order: the hardware deals consecutive blocks round-robin
  // over the XCDs, so neighbouring tiles of a plane would each fetch their
  // shared halo lines and partial cache lines into a different L2.  The
  // blocks are renumbered so that the tiles of a plane are consecutive on one
  // XCD (a bijection on the grid: XCD x takes ceil or floor of nblk / kXcds
  // consecutive logical blocks).
  const unsigned nblk = gridDim.x * gridDim.y, bid = blockIdx.x + gridDim.x * blockIdx.y;
  const unsigned xcd = bid % kXcds, kk = bid / kXcds, per = nblk / kXcds, rem = nblk % kXcds;
  const unsigned lid = xcd < rem ? xcd * (per + 1) + kk : rem * (per + 1) + (xcd - rem) * per + kk;
  const int bx = (int)(lid % gridDim.x), p = (int)(lid / gridDim.x);
  int e;
  if (!batch_entry(bt, p, e)) return;
  // the job's fields, read in one round before the exit and the mode lookup
  // branch on them
  const LvJob& J = jobs[ent_prob(e)];
  const int active = J.active, ntile = J.ntile[DIR];
  const LevelDev L = J.L;
  const int tile = J.tile[DIR], scratch_words = J.scratch[DIR];
  const int* const jmode = J.mode;
  for (const void* v : {(const void*)jmode, (const void*)J.u, (const void*)J.u2, (const void*)J.f, (const void*)L.ua,
                        (const void*)L.da, (const void*)L.Rr, (const void*)L.Ca, (const void*)L.wb, (const void*)L.ub,
                        (const void*)L.db, (const void*)L.Cb, (const void*)L.wr})
    pin_scalar(v);
  for (int v : {active, ntile, tile, scratch_words, L.na, L.nb}) pin_scalar(v);
  if (!active || bx >= ntile) return;
  const int slot = ent_slot(e);
  const int m = jmode ? jmode[slot] : slot;
  pin_scalar(m);  // resolved before the loads that index by it are issued
  const int na = L.na, nb = L.nb;
  // radial lines: u -> u2; polar lines: u2 -> u (a launch never reads what
  // another of its blocks writes)
  const auto u = gbl(static_cast<const V*>(DIR == 0 ? J.u : J.u2) + (size_t)slot * na * nb);
  const auto uo = gbl(static_cast<V*>(DIR == 0 ? J.u2 : J.u) + (size_t)slot * na * nb);
  const auto f = gbl(static_cast<const V*>(J.f) + (size_t)slot * na * nb);
  // tile geometry in (row, col) = (i, j) coordinates
  int r0, nr, c0, nc;  // first global row/col held in LDS and counts (incl. halo/pad)
  if (DIR == 1) {
    const int i0 = bx * tile;
    r0 = i0 - 2; nr = tile + 4;
    c0 = -1; nc = nb + 2;
  } else {
    // row stride odd (one unused column when tile + 4 is even): the lanes
    // walk down the columns
    const int j0 = bx * tile;
    r0 = -1; nr = na + 2;
    c0 = j0 - 2; nc = odd_stride(tile + 4);
  }
  const int ncu = DIR == 0 ? tile + 4 : nc;  // columns holding plane data
  V* fs = sh + nr * nc;  // staged f (SOR variant only)
  // line range of this tile (the coordinate across the lines)
  const int lbeg = bx * tile;                             // first owned line
  const int nlines_total = DIR == 1 ? na : nb;
  const int lend = min(lbeg + tile, nlines_total);        // one past the last owned line
  const int npts = DIR == 1 ? nb : na;                    // points per line
  const int fbeg = max(lbeg - 1, 0), fend = min(lend + 1, nlines_total);
  // LDS arrays after the tiles: exact-line scratch, then the 1D tables per
  // tile row rr = i - r0 (ua, da, R, Ca, omega of the polar line) and per
  // tile column cc = j - c0 (ub, db, Cb, omega of the radial line), then
  // (PROLONG) the prolongation indices and weights per tile row and column
  R* cp = reinterpret_cast<R*>(EXACT ? fs : fs + nr * nc);
  R* t0 = cp + scratch_words;
  R *t1 = t0 + nr, *t2 = t1 + nr, *t3 = t2 + nr, *t4 = t3 + nr;
  R *c1 = t4 + nr, *c2 = c1 + nc, *c3 = c2 + nc, *c4 = c3 + nc;
  int* pix = reinterpret_cast<int*>(c4 + nc);          // a0, a1 per row; b0, b1 per column
  R* pwt = reinterpret_cast<R*>(pix + 2 * (nr + nc));  // the matching weights
  const int par = m & 1;
  // Load phase.  The first batch (up to KB values of the u tile and of f per
  // thread, the thread's table row and column, and the prolongation tables)
  // is read into registers before anything is stored to LDS, so the block
  // waits for one round of memory latency rather than one per array; larger
  // tiles continue in strided loops.  The u tile is zero outside the plane.
  constexpr int KB = 4;
  const int n_u = nr * nc;
  const int fw = fend - fbeg;  // lines whose f is staged
  const int n_f = EXACT ? 0 : (DIR == 1 ? fw * nb : na * fw);
  auto u_pos = [&](int t, int& i, int& j) {
    const int rr = t / nc, cc = t - rr * nc;
    i = r0 + rr;
    j = c0 + cc;
    return cc < ncu && i >= 0 && i < na && j >= 0 && j < nb;
  };
  auto f_pos = [&](int t, int& i, int& j) {
    if (DIR == 1) {
      i = fbeg + t / nb;
      j = t % nb;
    } else {
      i = t / fw;
      j = fbeg + t % fw;
    }
  };
  V ub[KB], fb[KB];
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    const int t = threadIdx.x + k * NT;
    int i, j;
    ub[k] = mkv<R>(0, 0);
    if (!ZERO && t < n_u && u_pos(t, i, j)) ub[k] = u[(size_t)i * nb + j];
  }
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    const int t = threadIdx.x + k * NT;
    fb[k] = mkv<R>(0, 0);
    if (t < n_f) {
      int i, j;
      f_pos(t, i, j);
      fb[k] = f[(size_t)i * nb + j];
    }
  }
  // The table loads are unconditional (indices clamped into the plane) and
  // rows or columns outside it are masked arithmetically (x * 1 + 0 == x):
  // a select or a guard on a load becomes a branch that waits for the load
  // inside it, one round of memory latency per table.
  auto row_tables = [&](int rr, R* tr) {
    const int i = r0 + rr;
    const R in = (i >= 0 && i < na) ? (R)1 : (R)0;
    const int ic = min(max(i, 0), na - 1);
    const double a0 = gbl(L.ua)[ic], a1 = gbl(L.da)[ic], a2 = gbl(L.Rr)[ic];
    const double a3 = gbl(L.Ca)[(size_t)m * na + ic], a4 = gbl(L.wb)[(size_t)m * na + ic];
    tr[0] = (R)a0 * in;
    tr[1] = (R)a1 * in;
    tr[2] = (R)a2 * in;
    tr[3] = (R)a3 * in + ((R)1 - in);
    tr[4] = (R)a4 * in;
  };
  auto col_tables = [&](int cc, R* tc) {
    const int j = c0 + cc;
    const R in = (j >= 0 && j < nb) ? (R)1 : (R)0;
    const int jc = min(max(j, 0), nb - 1);
    const double b0 = gbl(L.ub)[jc], b1 = gbl(L.db)[jc];
    const double b2 = gbl(L.Cb)[(size_t)m * nb + jc], b3 = gbl(L.wr)[(size_t)m * nb + jc];
    tc[0] = (R)b0 * in;
    tc[1] = (R)b1 * in;
    tc[2] = (R)b2 * in;
    tc[3] = (R)b3 * in;
  };
  auto row_prolong = [&](int rr, int* ix, R* w) {
    const int i = min(max(r0 + rr, 0), na - 1);
    ix[0] = gbl(L.pa_i0)[i];
    ix[1] = gbl(L.pa_i1)[i];
    w[0] = (R)gbl(L.pa_w0)[i];
    w[1] = (R)gbl(L.pa_w1)[i];
  };
  auto col_prolong = [&](int cc, int* ix, R* w) {
    const int j = min(max(c0 + cc, 0), nb - 1);
    ix[0] = gbl(L.pb_i0)[par * nb + j];
    ix[1] = gbl(L.pb_i1)[par * nb + j];
    w[0] = (R)gbl(L.pb_w0)[par * nb + j];
    w[1] = (R)gbl(L.pb_w1)[par * nb + j];
  };
  auto store_row = [&](int rr, const R* tr, const int* ix, const R* w) {
    t0[rr] = tr[0]; t1[rr] = tr[1]; t2[rr] = tr[2]; t3[rr] = tr[3]; t4[rr] = tr[4];
    if (PROLONG) {
      pix[rr] = ix[0]; pix[nr + rr] = ix[1];
      pwt[rr] = w[0]; pwt[nr + rr] = w[1];
    }
  };
  auto store_col = [&](int cc, const R* tc, const int* ix, const R* w) {
    c1[cc] = tc[0]; c2[cc] = tc[1]; c3[cc] = tc[2]; c4[cc] = tc[3];
    if (PROLONG) {
      pix[2 * nr + cc] = ix[0]; pix[2 * nr + nc + cc] = ix[1];
      pwt[2 * nr + cc] = w[0]; pwt[2 * nr + nc + cc] = w[1];
    }
  };
  const int me = threadIdx.x;
  R tr[5], tc[4], wr[2] = {0, 0}, wc[2] = {0, 0};
  int ir[2] = {0, 0}, ic[2] = {0, 0};
  // every thread loads (clamped to the last row and column), so no load
  // sits behind a branch; only the owners store
  row_tables(min(me, nr - 1), tr);
  if (PROLONG) row_prolong(min(me, nr - 1), ir, wr);
  col_tables(min(me, nc - 1), tc);
  if (PROLONG) col_prolong(min(me, nc - 1), ic, wc);
  // stores of the first batch
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    const int t = threadIdx.x + k * NT;
    if (!PROLONG && t < n_u) sh[t] = ub[k];
  }
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    const int t = threadIdx.x + k * NT;
    if (t < n_f) {
      int i, j;
      f_pos(t, i, j);
      fs[(i - r0) * nc + (j - c0)] = fb[k];
    }
  }
  if (me < nr) store_row(me, tr, ir, wr);
  if (me < nc) store_col(me, tc, ic, wc);
  // the rest of larger tiles (reads clamped into the plane and masked, so
  // that the unrolled iterations' reads are in flight together)
  if (!PROLONG) {
#pragma unroll 4
    for (int t = threadIdx.x + KB * NT; t < n_u; t += NT) {
      int i, j;
      const R in = u_pos(t, i, j) ? (R)1 : (R)0;
      V v = mkv<R>(0, 0);
      if (!ZERO) v = u[(size_t)min(max(i, 0), na - 1) * nb + min(max(j, 0), nb - 1)];
      sh[t] = mkv<R>(v.x * in, v.y * in);
    }
  }
#pragma unroll 4
  for (int t = threadIdx.x + KB * NT; t < n_f; t += NT) {
    int i, j;
    f_pos(t, i, j);
    fs[(i - r0) * nc + (j - c0)] = f[(size_t)i * nb + j];
  }
  for (int rr = me + NT; rr < nr; rr += NT) {
    R tr2[5], w2[2] = {0, 0};
    int ix2[2] = {0, 0};
    row_tables(rr, tr2);
    if (PROLONG) row_prolong(rr, ix2, w2);
    store_row(rr, tr2, ix2, w2);
  }
  for (int cc = me + NT; cc < nc; cc += NT) {
    R tc2[4], w2[2] = {0, 0};
    int ix2[2] = {0, 0};
    col_tables(cc, tc2);
    if (PROLONG) col_prolong(cc, ix2, w2);
    store_col(cc, tc2, ix2, w2);
  }
  if constexpr (PROLONG) {
    // u tile plus the interpolated coarse correction, from the staged tables
    __syncthreads();
    const int cnb = J.C.nb;
    const auto uc = gbl(static_cast<const V*>(J.uc) + (size_t)slot * J.C.na * cnb);
    // The first batch's positions, whose u is in registers: the coarse
    // values are read unconditionally (the position clamped into the tile;
    // the staged indices are in range for every tile row and column) and
    // cells outside the plane are masked arithmetically, so the reads of
    // all positions are in flight together.  For a cell in the plane the
    // operations and their order are those of coarse_corr + add (k_prolong),
    // so a fused launch rounds exactly like the separate pass.
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const int t = min(threadIdx.x + k * NT, n_u - 1);
      const int rr = t / nc, cc = t - rr * nc;
      int i, j;
      const R in = u_pos(t, i, j) ? (R)1 : (R)0;
      const int a0 = pix[rr], a1 = pix[nr + rr], b0 = pix[2 * nr + cc], b1 = pix[2 * nr + nc + cc];
      const R wa0 = pwt[rr], wa1 = pwt[nr + rr], wb0 = pwt[2 * nr + cc], wb1 = pwt[2 * nr + nc + cc];
      V ev = mkv<R>(0, 0);
      ev = axpy<R>(wa0 * wb0, (V)uc[(size_t)a0 * cnb + b0], ev);
      ev = axpy<R>(wa0 * wb1, (V)uc[(size_t)a0 * cnb + b1], ev);
      ev = axpy<R>(wa1 * wb0, (V)uc[(size_t)a1 * cnb + b0], ev);
      ev = axpy<R>(wa1 * wb1, (V)uc[(size_t)a1 * cnb + b1], ev);
      ub[k] = mkv<R>((ub[k].x + ev.x) * in, (ub[k].y + ev.y) * in);
    }
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const int t = threadIdx.x + k * NT;
      if (t < n_u) sh[t] = ub[k];
    }
    // the rest of larger tiles, in the same form
#pragma unroll 4
    for (int t = threadIdx.x + KB * NT; t < n_u; t += NT) {
      const int rr = t / nc, cc = t - rr * nc;
      int i, j;
      const R in = u_pos(t, i, j) ? (R)1 : (R)0;
      const int a0 = pix[rr], a1 = pix[nr + rr], b0 = pix[2 * nr + cc], b1 = pix[2 * nr + nc + cc];
      const R wa0 = pwt[rr], wa1 = pwt[nr + rr], wb0 = pwt[2 * nr + cc], wb1 = pwt[2 * nr + nc + cc];
      V ev = mkv<R>(0, 0);
      ev = axpy<R>(wa0 * wb0, (V)uc[(size_t)a0 * cnb + b0], ev);
      ev = axpy<R>(wa0 * wb1, (V)uc[(size_t)a0 * cnb + b1], ev);
      ev = axpy<R>(wa1 * wb0, (V)uc[(size_t)a1 * cnb + b0], ev);
      ev = axpy<R>(wa1 * wb1, (V)uc[(size_t)a1 * cnb + b1], ev);
      const V w = u[(size_t)min(max(i, 0), na - 1) * nb + min(max(j, 0), nb - 1)];
      sh[t] = mkv<R>((w.x + ev.x) * in, (w.y + ev.y) * in);
    }
  }
  __syncthreads();
  const LineView<R> view{sh, nc, -r0, -c0, fs, nc, -r0, -c0, t0, t1, t2, t3, t4, -r0, c1, c2, c3, c4, -c0};
  for (int lc = 0; lc < 2; ++lc) {
    // colour lc: the first colour includes the inner halo lines
    int a = lc == 0 ? fbeg : lbeg;
    const int b = lc == 0 ? fend : lend;  // exclusive
    if ((a & 1) != lc) ++a;
    if (!EXACT) {
      relax_colour<DIR, PMAX, R>(view, a, b, npts, n_sor);
      __syncthreads();
      continue;
    }
    // Thomas algorithm along each line of the colour; the couplings to the
    // neighbouring lines (the other colour) are fixed right-hand-side terms.
    const int nl = a < b ? (b - a + 1) / 2 : 0;  // lines a, a+2, ... < b
    for (int t = threadIdx.x; t < nl; t += blockDim.x) {
      const int line = a + 2 * t;
      R* cpl = cp + t * npts;
      V prev = mkv<R>(0, 0);
      R cprev = 0;
      for (int k = 0; k < npts; ++k) {
        const int i = DIR == 1 ? line : k;
        const int j = DIR == 1 ? k : line;
        const int rr = i - r0, cc = j - c0;
        const R Rr = t2[rr];
        const R c = t3[rr] + Rr * c3[cc];
        R lo, up, w1, w2;
        V o1, o2;
        if (DIR == 1) {  // line along j; fixed neighbours i+1, i-1
          lo = Rr * c2[cc]; up = Rr * c1[cc];
          o1 = sh[(rr + 1) * nc + cc]; o2 = sh[(rr - 1) * nc + cc];
          w1 = t0[rr]; w2 = t1[rr];
        } else {         // line along i; fixed neighbours j+1, j-1
          lo = t1[rr]; up = t0[rr];
          o1 = sh[rr * nc + cc + 1]; o2 = sh[rr * nc + cc - 1];
          w1 = Rr * c1[cc]; w2 = Rr * c2[cc];
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
  }
  // write back the owned lines (ACC: add them to the FP64 iterate instead)
  if constexpr (ACC) {
    const auto a = gbl(J.acc + (size_t)slot * na * nb);
#pragma unroll 4
    for (int t = threadIdx.x; t < (lend - lbeg) * nb; t += blockDim.x) {
      const int i = lbeg + t / nb, j = t % nb;
      const V ev = sh[(i - r0) * nc + (j - c0)];
      const double2 v = a[(size_t)i * nb + j];
      a[(size_t)i * nb + j] = make_double2(v.x + (double)ev.x, v.y + (double)ev.y);
    }
  } else if (DIR == 1) {
    for (int t = threadIdx.x; t < (lend - lbeg) * nb; t += blockDim.x) {
      const int i = lbeg + t / nb, j = t % nb;
      uo[(size_t)i * nb + j] = sh[(i - r0) * nc + (j - c0)];
    }
  } else {
    const int w = lend - lbeg;
    for (int t = threadIdx.x; t < na * w; t += blockDim.x) {
      const int i = t / w, j = lbeg + t % w;
      uo[(size_t)i * nb + j] = sh[(i - r0) * nc + (j - c0)];
    }
  }
}

// Common prologue of the per-cell kernels: resolve list entry blockIdx.y.
#define SMG_ENTRY(JOBS, BT)                                  \
  const int p = blockIdx.y;                                  \
  int e;                                                     \
  if (!batch_entry((BT), p, e)) return;                      \
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
// coarse correction starts from zero.  A thread reads everything its coarse
// cell needs (the 2 x 2 fine cells' stencils of u, f, the row and column
// tables and the restriction weights) before it computes, so one round of
// memory latency covers them; the residuals are those of resid_at, with the
// same operations in the same order.
template <typename R>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(1, 4)))
k_restrict(const LvJob* __restrict__ jobs, BatchRef bt) {
  using V = typename Vec<R>::T;
  SMG_ENTRY(jobs, bt);
  if (!J.active) return;
  const LevelDev L = J.L, C = J.C;
  const size_t off = (size_t)slot * L.na * L.nb;
  const size_t offc = (size_t)slot * C.na * C.nb;
  const auto U = gbl(static_cast<const V*>(J.u) + off);
  const auto F = gbl(static_cast<const V*>(J.f) + off);
  const auto FC = gbl(static_cast<V*>(J.fc) + offc);
  const auto UC = gbl(static_cast<V*>(J.uc) + offc);
  const int na = L.na, nb = L.nb;
  const int cells = C.na * C.nb;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < cells; t += gridDim.x * blockDim.x) {
    const int I = t / C.nb, Jc = t - I * C.nb;
    R wa[2], wb[2], Rr[2], ca[2], ua[2], da[2], cb[2], ub[2], db[2];
    V uc[2][2], uip[2][2], uim[2][2], ujp[2][2], ujm[2][2], fv[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int i = 2 * I + a;
      wa[a] = (R)gbl(L.rwa)[i];
      Rr[a] = (R)gbl(L.Rr)[i];
      ca[a] = (R)gbl(L.Ca)[(size_t)m * na + i];
      ua[a] = (R)gbl(L.ua)[i];
      da[a] = (R)gbl(L.da)[i];
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int j = 2 * Jc + b;
      wb[b] = (R)gbl(L.rwb)[j];
      cb[b] = (R)gbl(L.Cb)[(size_t)m * nb + j];
      ub[b] = (R)gbl(L.ub)[j];
      db[b] = (R)gbl(L.db)[j];
    }
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int i = 2 * I + a;
      const int ip = min(i + 1, na - 1), im = max(i - 1, 0);
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int j = 2 * Jc + b;
        const int jp = min(j + 1, nb - 1), jm = max(j - 1, 0);
        const size_t row = (size_t)i * nb;
        uc[a][b] = U[row + j];
        uip[a][b] = U[(size_t)ip * nb + j];
        uim[a][b] = U[(size_t)im * nb + j];
        ujp[a][b] = U[row + jp];
        ujm[a][b] = U[row + jm];
        fv[a][b] = F[row + j];
      }
    }
    V acc = mkv<R>(0, 0);
#pragma unroll
    for (int a = 0; a < 2; ++a) {
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const R w = wa[a] * wb[b];
        const R c = ca[a] + Rr[a] * cb[b];
        V s = mkv<R>(c * uc[a][b].x, c * uc[a][b].y);
        s = axpy<R>(ua[a], uip[a][b], s);
        s = axpy<R>(da[a], uim[a][b], s);
        s = axpy<R>(Rr[a] * ub[b], ujp[a][b], s);
        s = axpy<R>(Rr[a] * db[b], ujm[a][b], s);
        const V r = mkv<R>(fv[a][b].x - s.x, fv[a][b].y - s.y);
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
  const auto U = gbl(static_cast<V*>(J.u) + (size_t)slot * L.na * L.nb);
  const auto uc = gbl(static_cast<const V*>(J.uc) + (size_t)slot * C.na * C.nb);
  const int par = m & 1;
  const int cells = L.na * L.nb;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < cells; t += gridDim.x * blockDim.x) {
    const int i = t / L.nb, j = t - i * L.nb;
    const V ev = coarse_corr<R>(L, C.nb, uc, par, i, j);
    const V v = U[t];
    U[t] = mkv<R>(v.x + ev.x, v.y + ev.y);
  }
}

// Volume-weighted squared defect (FP64): partial sums per (list position,
// block).  use_u = 0: the defect of the zero guess (f itself).  With the
// mixed form the FP64 residual is also stored rounded to FP32 (the right-hand
// side of the next FP32 correction cycle) and (zero_e) the FP32 correction is
// zeroed; with norm_only neither (the zero-guess norm of a warm start, whose
// own defect pass writes them next).  With zero_u (zero guess only) the FP64
// iterate is set to zero as well, in place of a separate fill.
__global__ void __launch_bounds__(kThreads) k_norm_partial(const NormJob* __restrict__ jobs, BatchRef bt, int use_u,
                                                          double* __restrict__ partial, int zero_e, int zero_u,
                                                          int norm_only) {
  __shared__ double red[kThreads / 64];
  SMG_ENTRY(jobs, bt);
  const LevelDev L = J.L;
  const size_t off = (size_t)slot * L.na * L.nb;
  const double2* U = J.u + off;
  const double2* F = J.f + off;
  const auto R32 = gbl(J.r32 && !norm_only ? J.r32 + off : nullptr);
  const auto E32 = gbl(J.e32 ? J.e32 + off : nullptr);
  const int cells = L.na * L.nb;
  double acc = 0.0;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < cells; t += gridDim.x * blockDim.x) {
    const int i = t / L.nb, j = t - i * L.nb;
    const double2 r = use_u ? resid_at<double>(L, m, U, F, i, j) : (double2)gbl(F)[t];
    if (zero_u) gbl(J.u + off)[t] = make_double2(0.0, 0.0);  // zero guess: u starts at 0
    if (R32) {
      R32[t] = make_float2((float)r.x, (float)r.y);
      if (zero_e) E32[t] = make_float2(0.f, 0.f);
    }
    acc += (r.x * r.x + r.y * r.y) * (gbl(L.va)[i] * gbl(L.vb)[j]);
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
  const auto U = gbl(J.u + off);
  const auto E = gbl(J.e32 + off);
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


}  // namespace

namespace smgk {

size_t lds_limit() {
  static size_t cached[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 64 * 1024;
  if (!cached[dev]) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v < 64 * 1024)
      v = 64 * 1024;
    cached[dev] = (size_t)v;
  }
  return cached[dev];
}

// Lines per tile so that a launch over `planes` planes has about
// target_blocks blocks, within the LDS budget.
bool smooth_shape(const LevelDev& L, int dir, bool exact, bool fp32, int target_blocks, int planes, SmoothShape* out) {
  const int npts = dir == 0 ? L.na : L.nb;    // points per line
  const int nlines = dir == 0 ? L.nb : L.na;  // lines in the plane
  if (npts > kRelaxMaxPoints) return false;
  auto bytes = [&](int t) {
    const int scratch = exact ? (t / 2 + 2) * npts : 0;
    return fp32 ? smooth_lds_bytes<float>(dir, L.na, L.nb, t, exact, scratch)
                : smooth_lds_bytes<double>(dir, L.na, L.nb, t, exact, scratch);
  };
  if (planes < 1) planes = 1;
  const int want = (target_blocks + planes - 1) / planes;  // tiles per plane
  int tile = (nlines + want - 1) / want;
  if (tile < 2) tile = 2;
  if (tile > nlines) tile = nlines;
  while (tile > 2 && bytes(tile) > lds_limit() - 1024) --tile;
  if (tile > 2 && (tile & 1)) --tile;
  out->tile = tile;
  out->ntile = (nlines + tile - 1) / tile;
  out->scratch = exact ? (tile / 2 + 2) * npts : 0;
  out->lds = bytes(tile);
  return out->lds <= lds_limit();
}

static thread_local hipEvent_t t_ev_start = nullptr, t_ev_stop = nullptr;

void next_launch_events(hipEvent_t start, hipEvent_t stop) {
  t_ev_start = start;
  t_ev_stop = stop;
}

template <typename R>
static hipError_t smooth_launch(const LvJob* jobs, const LvJob* hj, int n_prob, const BatchRef& b, int n_sor,
                                bool exact, int dir, int in, bool acc, hipStream_t st) {
  const bool prolong = in == kInProlong;
  int gx = 0;
  size_t lds = 0;
  for (int q = 0; q < n_prob; ++q) {
    if (!hj[q].active) continue;
    const LevelDev& L = hj[q].L;
    if ((dir == 0 ? L.na : L.nb) > kRelaxMaxPoints) return hipErrorInvalidConfiguration;
    lds = std::max(lds, smooth_lds_bytes<R>(dir, L.na, L.nb, hj[q].tile[dir], exact, hj[q].scratch[dir], prolong));
    if (hj[q].ntile[dir] > gx) gx = hj[q].ntile[dir];
  }
  if (gx == 0 || b.cap == 0) return hipSuccess;
  if (prolong && lds > lds_limit()) {
    // the tables do not fit beside the widest tile: separate prolongation
    hipError_t e = mg_prolong(jobs, hj, n_prob, b, std::is_same<R, float>::value, st);
    if (e != hipSuccess) return e;
    return smooth_launch<R>(jobs, hj, n_prob, b, n_sor, exact, dir, kInLoad, acc, st);
  }
  if (lds > lds_limit()) return hipErrorInvalidConfiguration;
  const dim3 grid(gx, b.cap);
  // Block size: enough waves to relax the first colour's lines (tile / 2
  // owned lines of one parity and the inner halo line) in one step, 256,
  // 512 or 1024 threads; 512 and 1024 only for lines of up to 4 points per
  // lane, where the variant stays within 128 registers.
  int pmax = 2, waves = 1;
  for (int q = 0; q < n_prob; ++q)
    if (hj[q].active) {
      const int npts = dir == 0 ? hj[q].L.na : hj[q].L.nb;
      const int P = relax_points_per_lane(npts);
      const int per_wave = 64 / ((npts + P - 1) / P);  // lines a wave relaxes at once
      pmax = std::max(pmax, P);
      waves = std::max(waves, (hj[q].tile[dir] / 2 + 1 + per_wave - 1) / per_wave);
    }
  const int nt = exact || pmax > 4 || waves <= 4 ? 256 : (waves <= 8 ? 512 : 1024);
  // the coarse correction is applied by radial-line launches only, the
  // accumulation into the FP64 iterate by FP32 polar-line launches only
  if (in != kInLoad && dir != 0) return hipErrorInvalidValue;
  if (acc && (dir != 1 || !std::is_same<R, float>::value)) return hipErrorInvalidValue;
  for (int q = 0; q < n_prob; ++q) {
    if (acc && hj[q].active && !hj[q].acc) return hipErrorInvalidValue;
    if (hj[q].active && (!hj[q].u || !hj[q].u2)) return hipErrorInvalidValue;
  }
  auto go = [&](auto kern, int nt) {
    if (t_ev_start) {
      hipExtLaunchKernelGGL(kern, grid, dim3(nt), lds, st, t_ev_start, t_ev_stop, 0u, jobs, b, n_sor);
      t_ev_start = t_ev_stop = nullptr;
    } else {
      hipLaunchKernelGGL(kern, grid, dim3(nt), lds, st, jobs, b, n_sor);
    }
  };
  // radial launch with or without the coarse correction; polar launch
  // storing the lines or adding them to the FP64 iterate
  auto go0 = [&](auto kern_plain, auto kern_prolong, auto kern_zero, int nt) {
    in == kInProlong ? go(kern_prolong, nt) : (in == kInZero ? go(kern_zero, nt) : go(kern_plain, nt));
  };
  auto go1 = [&](auto kern_plain, auto kern_acc, int nt) { acc ? go(kern_acc, nt) : go(kern_plain, nt); };
  if (exact) {
    if (dir == 0) go0(k_smooth<0, true, 2, R, kThreads, kInLoad>, k_smooth<0, true, 2, R, kThreads, kInProlong>, k_smooth<0, true, 2, R, kThreads, kInZero>, kThreads);
    else go1(k_smooth<1, true, 2, R, kThreads, kInLoad>, k_smooth<1, true, 2, R, kThreads, kInLoad, true>, kThreads);
  } else if (nt == 1024) {
    if (dir == 0) {
      if (pmax <= 2) go0(k_smooth<0, false, 2, R, 1024, kInLoad>, k_smooth<0, false, 2, R, 1024, kInProlong>, k_smooth<0, false, 2, R, 1024, kInZero>, 1024);
      else go0(k_smooth<0, false, 4, R, 1024, kInLoad>, k_smooth<0, false, 4, R, 1024, kInProlong>, k_smooth<0, false, 4, R, 1024, kInZero>, 1024);
    } else {
      if (pmax <= 2) go1(k_smooth<1, false, 2, R, 1024, kInLoad>, k_smooth<1, false, 2, R, 1024, kInLoad, true>, 1024);
      else go1(k_smooth<1, false, 4, R, 1024, kInLoad>, k_smooth<1, false, 4, R, 1024, kInLoad, true>, 1024);
    }
  } else if (nt == 512) {
    if (dir == 0) {
      if (pmax <= 2) go0(k_smooth<0, false, 2, R, 512, kInLoad>, k_smooth<0, false, 2, R, 512, kInProlong>, k_smooth<0, false, 2, R, 512, kInZero>, 512);
      else go0(k_smooth<0, false, 4, R, 512, kInLoad>, k_smooth<0, false, 4, R, 512, kInProlong>, k_smooth<0, false, 4, R, 512, kInZero>, 512);
    } else {
      if (pmax <= 2) go1(k_smooth<1, false, 2, R, 512, kInLoad>, k_smooth<1, false, 2, R, 512, kInLoad, true>, 512);
      else go1(k_smooth<1, false, 4, R, 512, kInLoad>, k_smooth<1, false, 4, R, 512, kInLoad, true>, 512);
    }
  } else if (dir == 0) {
    if (pmax <= 2) go0(k_smooth<0, false, 2, R, kThreads, kInLoad>, k_smooth<0, false, 2, R, kThreads, kInProlong>, k_smooth<0, false, 2, R, kThreads, kInZero>, kThreads);
    else if (pmax <= 4) go0(k_smooth<0, false, 4, R, kThreads, kInLoad>, k_smooth<0, false, 4, R, kThreads, kInProlong>, k_smooth<0, false, 4, R, kThreads, kInZero>, kThreads);
    else if (pmax <= 8) go0(k_smooth<0, false, 8, R, kThreads, kInLoad>, k_smooth<0, false, 8, R, kThreads, kInProlong>, k_smooth<0, false, 8, R, kThreads, kInZero>, kThreads);
    else go0(k_smooth<0, false, 16, R, kThreads, kInLoad>, k_smooth<0, false, 16, R, kThreads, kInProlong>, k_smooth<0, false, 16, R, kThreads, kInZero>, kThreads);
  } else {
    if (pmax <= 2) go1(k_smooth<1, false, 2, R, kThreads, kInLoad>, k_smooth<1, false, 2, R, kThreads, kInLoad, true>, kThreads);
    else if (pmax <= 4) go1(k_smooth<1, false, 4, R, kThreads, kInLoad>, k_smooth<1, false, 4, R, kThreads, kInLoad, true>, kThreads);
    else if (pmax <= 8) go1(k_smooth<1, false, 8, R, kThreads, kInLoad>, k_smooth<1, false, 8, R, kThreads, kInLoad, true>, kThreads);
    else go1(k_smooth<1, false, 16, R, kThreads, kInLoad>, k_smooth<1, false, 16, R, kThreads, kInLoad, true>, kThreads);
  }
  return hipGetLastError();
}

hipError_t mg_smooth_dir(const LvJob* jobs, const LvJob* hj, int n_prob, const BatchRef& b, int n_sor, bool exact,
                         int dir, bool fp32, hipStream_t st, bool prolong, bool accumulate, bool zero) {
  const int in = prolong ? kInProlong : (zero ? kInZero : kInLoad);
  if (prolong && zero) return hipErrorInvalidValue;
  return fp32 ? smooth_launch<float>(jobs, hj, n_prob, b, n_sor, exact, dir, in, accumulate, st)
              : smooth_launch<double>(jobs, hj, n_prob, b, n_sor, exact, dir, in, accumulate, st);
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
                           double* partial, int nblk, hipStream_t st, bool zero_e, bool zero_u, bool norm_only) {
  (void)hj; (void)n_prob;
  if (!b.cap) return hipSuccess;
  if (zero_u && use_u) return hipErrorInvalidValue;  // the defect of a guess it would erase
  hipLaunchKernelGGL(k_norm_partial, dim3(nblk, b.cap), dim3(kThreads), 0, st, jobs, b, use_u ? 1 : 0, partial,
                     zero_e ? 1 : 0, zero_u ? 1 : 0, norm_only ? 1 : 0);
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
