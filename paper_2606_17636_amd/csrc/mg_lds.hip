// The coarse end of the V-cycle in one launch: every level whose plane fits
// in LDS (from level `first` down to the coarsest) is processed by one block
// per plane -- pre-smoothing, residual restriction, the coarsest solve,
// prolongation and post-smoothing -- without touching global memory between
// levels.  The coarsest level is solved exactly by fast diagonalisation
// where the host built its tables (row transforms on the FP64 matrix cores,
// tridiagonal sweeps in segments), else by red-black SOR (Sec. 3.3).  The arithmetic is that of the per-level kernels in
// mg.hip (same colour order, same transfer weights, same stopping rule of
// the coarsest solve); only the memory traffic and the launch count differ.
// Templated on the real type R of the smoothing levels; the coarsest level
// is always solved in FP64 (the mixed form keeps the coarsest solve in FP64).
#include <algorithm>

#include "batch_dev.h"
#include "relax_dev.h"
#include "smg_internal.h"
#include "vec.h"

namespace {

constexpr int kAliasCells = 4;  // coarse cells per thread of the aliased restriction

// Row strides of a smoothed level's padded u and of its f (odd: see
// odd_stride); the coarsest level keeps nb + 2 and nb.
__host__ __device__ __forceinline__ int lvl_us(int nb) { return odd_stride(nb + 2); }
__host__ __device__ __forceinline__ int lvl_fs(int nb) { return odd_stride(nb); }

struct Red {
  double* buf;
  __device__ double sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) buf[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += buf[w];
    return s;
  }
};

// 1D stencil tables of one level and mode, staged in LDS (rounded to R).
template <typename R>
struct Tab {
  const R *ua, *da, *Rr, *Ca, *wb;  // per row i
  const R *ub, *db, *Cb, *wr;       // per column j
};

template <typename R>
__device__ __forceinline__ Tab<R> tab_at(R* t, int na, int nb) {
  R* c = t + 5 * na;
  return Tab<R>{t, t + na, t + 2 * na, t + 3 * na, t + 4 * na, c, c + nb, c + 2 * nb, c + 3 * nb};
}

template <typename R>
__device__ __forceinline__ Tab<R> stage_tab(const LevelDev& L, int m, R* buf) {
  const int na = L.na, nb = L.nb;
  R* t = buf;
  for (int i = threadIdx.x; i < na; i += blockDim.x) {
    t[i] = (R)gbl(L.ua)[i];
    t[na + i] = (R)gbl(L.da)[i];
    t[2 * na + i] = (R)gbl(L.Rr)[i];
    t[3 * na + i] = (R)gbl(L.Ca)[(size_t)m * na + i];
    t[4 * na + i] = (R)gbl(L.wb)[(size_t)m * na + i];
  }
  R* c = buf + 5 * na;
  for (int j = threadIdx.x; j < nb; j += blockDim.x) {
    c[j] = (R)gbl(L.ub)[j];
    c[nb + j] = (R)gbl(L.db)[j];
    c[2 * nb + j] = (R)gbl(L.Cb)[(size_t)m * nb + j];
    c[3 * nb + j] = (R)gbl(L.wr)[(size_t)m * nb + j];
  }
  return tab_at<R>(buf, na, nb);
}

// One zebra phase in direction DIR (0: radial lines, fixed j, points along
// i; 1: polar lines, fixed i, points along j): the lines of colour 0, then
// those of colour 1, each line relaxed by n_sor even-odd SOR passes in
// registers; one barrier separates the colours.
// u: padded (na+2) x (nb+2) plane, f: na x nb.
template <int DIR, int PMAX, typename R>
__device__ __forceinline__ void sor_phase(const LevelDev& L, const Tab<R>& T, typename Vec<R>::T* u, const typename Vec<R>::T* f,
                          int n_sor) {
  const int na = L.na, nb = L.nb;
  const LineView<R> v{u, lvl_us(nb), 1, 1, f, lvl_fs(nb), 0, 0, T.ua, T.da, T.Rr, T.Ca, T.wb, 0, T.ub, T.db, T.Cb, T.wr, 0};
  const int npts = DIR == 0 ? na : nb, nlines = DIR == 0 ? nb : na;
  for (int lc = 0; lc < 2; ++lc) {
    relax_colour<DIR, PMAX, R>(v, lc, nlines, npts, n_sor);
    __syncthreads();
  }
}

template <int DIR, typename R>
__device__ __forceinline__ void exact_phase(const LevelDev& L, const Tab<R>& T, typename Vec<R>::T* u, const typename Vec<R>::T* f,
                            R* cp) {
  using V = typename Vec<R>::T;
  const int na = L.na, nb = L.nb, nc = lvl_us(nb), fs = lvl_fs(nb);
  const int npts = DIR == 0 ? na : nb;
  for (int lc = 0; lc < 2; ++lc) {
    const int nl = DIR == 0 ? (nb - lc + 1) / 2 : (na - lc + 1) / 2;
    for (int t = threadIdx.x; t < nl; t += blockDim.x) {
      const int line = lc + 2 * t;
      R* c1 = cp + t * npts;
      V prev = mkv<R>(0, 0);
      R cprev = 0;
      for (int k = 0; k < npts; ++k) {
        const int i = DIR == 1 ? line : k, j = DIR == 1 ? k : line;
        const int q = (i + 1) * nc + (j + 1);
        const R Rr = T.Rr[i];
        const R c = T.Ca[i] + Rr * T.Cb[j];
        R lo, up, w1, w2;
        V o1, o2;
        if (DIR == 1) {
          lo = Rr * T.db[j]; up = Rr * T.ub[j];
          o1 = u[q + nc]; o2 = u[q - nc]; w1 = T.ua[i]; w2 = T.da[i];
        } else {
          lo = T.da[i]; up = T.ua[i];
          o1 = u[q + 1]; o2 = u[q - 1]; w1 = Rr * T.ub[j]; w2 = Rr * T.db[j];
        }
        const V fv = f[i * fs + j];
        const R rx = fv.x - (w1 * o1.x + w2 * o2.x), ry = fv.y - (w1 * o1.y + w2 * o2.y);
        const R den = c - lo * cprev;
        cprev = up / den;
        c1[k] = cprev;
        prev = mkv<R>((rx - lo * prev.x) / den, (ry - lo * prev.y) / den);
        u[q] = prev;
      }
      for (int k = npts - 2; k >= 0; --k) {
        const int i = DIR == 1 ? line : k, j = DIR == 1 ? k : line;
        const int q = (i + 1) * nc + (j + 1);
        const V nx = DIR == 1 ? u[q + 1] : u[q + nc];
        const V d = u[q];
        u[q] = mkv<R>(d.x - c1[k] * nx.x, d.y - c1[k] * nx.y);
      }
    }
    __syncthreads();
  }
}

template <int PMAX, typename R>
__device__ __forceinline__ void smooth_step(const LevelDev& L, const Tab<R>& T, typename Vec<R>::T* u, const typename Vec<R>::T* f,
                            int n_sor, bool exact, R* cp) {
  if (exact) {
    exact_phase<0, R>(L, T, u, f, cp);
    exact_phase<1, R>(L, T, u, f, cp);
  } else {
    sor_phase<0, PMAX, R>(L, T, u, f, n_sor);
    sor_phase<1, PMAX, R>(L, T, u, f, n_sor);
  }
}

// nc, fs: row strides of u (padded) and f
template <typename R>
__device__ __forceinline__ typename Vec<R>::T resid_lds(const LevelDev& L, const Tab<R>& T, const typename Vec<R>::T* u,
                                                        const typename Vec<R>::T* f, int i, int j, int nc, int fs) {
  const int q = (i + 1) * nc + (j + 1);
  const R Rr = T.Rr[i];
  const R c = T.Ca[i] + Rr * T.Cb[j];
  const R a1 = T.ua[i], a2 = T.da[i], b1 = Rr * T.ub[j], b2 = Rr * T.db[j];
  const auto un = u[q + nc], us = u[q - nc], ue = u[q + 1], uw = u[q - 1], uc = u[q];
  const auto fv = f[i * fs + j];
  return mkv<R>(fv.x - (c * uc.x + a1 * un.x + a2 * us.x + b1 * ue.x + b2 * uw.x),
                fv.y - (c * uc.y + a1 * un.y + a2 * us.y + b1 * ue.y + b2 * uw.y));
}

// Exact solve of the coarsest level by fast diagonalisation, in place on f
// ([na][nb] FP64 complex in LDS): rows w = f V^-T, then for every
// eigenvalue q the tridiagonal system along a by the Thomas factors (one
// lane per (q, real/imaginary part), the column held in registers in
// chunks), then rows u = w V^T.  The eigenvector tables sit in LDS from the
// start of the kernel (vt: V^T at [q][j], V^-T at [j][q] after it); the
// Thomas factors are staged into LDS (fac) here, all loads in flight at once.
constexpr int kSepChunk = 8;
// Segments per tridiagonal system in the exact coarse solve: a function of
// the level's width only (not of the block size), so that every launch shape
// rounds alike; about 512 (system, segment) pairs, at most 16 segments.  The
// segment-end scratch (forward and backward) takes 6 sep_seg_max(nb) nb
// doubles.
__host__ __device__ constexpr int sep_seg_max(int nb) { return nb >= 256 ? 1 : (nb >= 16 ? 256 / nb : 16); }

// Row transform of the exact coarse solve on the FP64 matrix cores:
// x[i][c] <- sum_r M[r][c] x[i][r] for every row i (M real, in LDS).  The
// plane x (LDS, row stride ws doubles) is either complex (QS = 1: the
// components interleaved, ws = 2 nb), whose rows split into real rows
// rho = 2 i + component, or one real component (QS = 0), so the transform is
// a real ((na << QS) x nb) by (nb x nb) product.  A wave
// owns 16 real rows (8 complex rows) and all columns: one accumulator per
// 16-column tile, K in steps of 4, one v_mfma_f64_16x16x4 per (tile, step).
// Operand layout of that instruction: lane l holds A[l % 16][l / 16] and
// B[l / 16][l % 16]; element e of its result is D[4 e + l / 16][l % 16].
// Rows, columns and K beyond the sizes are zero operands and are not
// written.  The wave has read all of its rows (its own LDS reads complete in
// order) before it writes them, and no other wave touches them, so the
// transform runs in place.
typedef double sep_d4 __attribute__((ext_vector_type(4)));
constexpr int kSepMaxTiles = 8;  // nb <= 128 (the host builds no tables beyond)

// NB > 0: the width as a compile-time constant, a multiple of 16: the K loop
// is unrolled whole, so no accumulator is carried around a loop (which would
// move it between register files at every step), and every operand read is
// in range with no select (rows beyond the plane read row 0 and feed only
// outputs that are not written).  NB = 0: any width, runtime K loop,
// operands beyond the sizes replaced by zero.
template <int QS, int NCT, int NB>
__device__ __forceinline__ void sep_rows_t(double* X, int na, int nb_rt, int ws, const double* M) {
  const int nb = NB ? NB : nb_rt;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
  const int lm = lane & 15, lk = lane >> 4;
  const int nrow = na << QS, nrb = (nrow + 15) >> 4;
  for (int rb = wave; rb < nrb; rb += nwave) {  // uniform in the wave
    const int rho_a = rb * 16 + lm;
    const bool row_ok = rho_a < nrow;
    const int abase = row_ok ? (rho_a >> QS) * ws + (rho_a & QS) : 0;
    int cc[NCT];
    bool c_ok[NCT];
#pragma unroll
    for (int t = 0; t < NCT; ++t) {
      const int c = t * 16 + lm;
      c_ok[t] = c < nb;
      cc[t] = c_ok[t] ? c : 0;
    }
    sep_d4 acc[NCT];
#pragma unroll
    for (int t = 0; t < NCT; ++t) acc[t] = (sep_d4){0.0, 0.0, 0.0, 0.0};
    if constexpr (NB > 0) {
#pragma unroll
      for (int k0 = 0; k0 < NB; k0 += 4) {
        const int r = k0 + lk;
        const double av = X[abase + (r << QS)];
#pragma unroll
        for (int t = 0; t < NCT; ++t)
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, M[r * NB + t * 16 + lm], acc[t], 0, 0, 0);
      }
    } else {
#pragma unroll 4
      for (int k0 = 0; k0 < nb; k0 += 4) {
        const int r = k0 + lk;
        const bool k_ok = r < nb;
        const int rr = k_ok ? r : 0;
        const double ax = X[abase + (rr << QS)];
        const double av = row_ok && k_ok ? ax : 0.0;
        double bv[NCT];
#pragma unroll
        for (int t = 0; t < NCT; ++t) {
          const double bx = M[rr * nb + cc[t]];
          bv[t] = k_ok && c_ok[t] ? bx : 0.0;
        }
#pragma unroll
        for (int t = 0; t < NCT; ++t) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[t], acc[t], 0, 0, 0);
      }
    }
#pragma unroll
    for (int t = 0; t < NCT; ++t) {
      const int c = t * 16 + lm;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int rho = rb * 16 + 4 * e + lk;
        if (rho < nrow && c < nb) X[(rho >> QS) * ws + (c << QS) + (rho & QS)] = acc[t][e];
      }
    }
  }
}

// The tile count as a compile-time constant (rounded up to a power of two;
// the extra tiles multiply zeros), and the usual widths fully unrolled.
template <int QS>
__device__ __forceinline__ void sep_rows(double* X, int na, int nb, int ws, const double* M) {
  const int nct = (nb + 15) >> 4;
  if (nb == 16) sep_rows_t<QS, 1, 16>(X, na, nb, ws, M);
  else if (nb == 32) sep_rows_t<QS, 2, 32>(X, na, nb, ws, M);
  else if (nb == 64) sep_rows_t<QS, 4, 64>(X, na, nb, ws, M);
  else if (nct <= 1) sep_rows_t<QS, 1, 0>(X, na, nb, ws, M);
  else if (nct <= 2) sep_rows_t<QS, 2, 0>(X, na, nb, ws, M);
  else if (nct <= 4) sep_rows_t<QS, 4, 0>(X, na, nb, ws, M);
  else sep_rows_t<QS, kSepMaxTiles, 0>(X, na, nb, ws, M);
}

// The exact coarse solve on a plane in LDS, in place: complex interleaved
// (QS = 1, ws = 2 nb) or one real component with row stride ws (QS = 0).
template <int QS>
__device__ __forceinline__ void coarse_separable(const LevelDev& L, const Tab<double>& T, int m, double* w, int ws,
                                                 const double* vt, double* fac, bool staged) {
  const int na = L.na, nb = L.nb, nn = na * nb;
  if (!staged) {
    const auto gcp = gbl(L.sep_cp + (size_t)m * nn), gid = gbl(L.sep_id + (size_t)m * nn);
#pragma unroll 4
    for (int t = threadIdx.x; t < nn; t += blockDim.x) {
      fac[t] = gcp[t];
      fac[nn + t] = gid[t];
    }
  }
  sep_rows<QS>(w, na, nb, ws, vt + nb * nb);
  __syncthreads();
  // Tridiagonal solves along a, one per (q, component): the forward sweep
  // y_i = id_i w_i - id_i da_i y_{i-1} and the back substitution
  // x_i = y_i - cp_i x_{i+1} are first-order linear recurrences.  Each
  // system's rows are cut into S segments; a thread solves its segment from
  // a zero carry while it multiplies up the recurrence coefficients, then,
  // after a barrier, takes the true value entering its segment from the
  // segment ends before it and adds carry * (coefficient product) to its
  // rows.  Lanes run over l = (q << QS) + component, so row i of every
  // system is the contiguous run w[i ws + l].
  const double* cp = fac;
  const double* id = fac + nn;
  const int nsys = nb << QS;
  int S = min(sep_seg_max(nb), na);
  const int len = (na + S - 1) / S;
  S = (na + len - 1) / len;
  double* pend = fac + 2 * nn;     // [S][nb] coefficient product of a segment
  double* eend = pend + S * nb;    // [S][2 nb] local value at the segment's far end
  double* pendB = eend + S * nsys; // the same for the back substitution
  double* eendB = pendB + S * nb;
  constexpr int kSegReg = 8;       // segment rows held in registers
  constexpr int kSegMax = 16;      // sep_seg_max never exceeds it
  if (len <= kSegReg && nsys * S <= (int)blockDim.x) {
    // One (system, segment) per thread, its rows in registers through both
    // sweeps: load once; forward from a zero carry; barrier; forward carry
    // and fix, then the back substitution from a zero carry, with no barrier
    // between them (the backward segment ends go to their own scratch);
    // barrier; backward carry and fix; store once.  Same operations in the
    // same order as the general path below.
    const int t = threadIdx.x;
    const bool act = t < nsys * S;
    const int l = act ? t % nsys : 0, sg = act ? t / nsys : 0, q = l >> QS;
    const int beg = sg * len, cnt = act ? min(na, beg + len) - beg : 0;
    double y[kSegReg], bf[kSegReg], bb[kSegReg];
    double yl = 0.0, P = 1.0;
#pragma unroll
    for (int k = 0; k < kSegReg; ++k) {
      const int i = beg + min(k, max(cnt - 1, 0));  // clamped into the segment
      const double wv = w[i * ws + l], iv = id[i * nb + q];
      const double dv = i > 0 ? T.da[i] : 0.0;
      const double cv = i < na - 1 ? cp[i * nb + q] : 0.0;
      const double a = wv * iv;
      bf[k] = -dv * iv;
      bb[k] = -cv;
      if (k < cnt) {
        yl = fma(bf[k], yl, a);
        P *= bf[k];
      }
      y[k] = yl;
    }
    if (act && S > 1) {
      if ((l & QS) == 0) pend[sg * nb + q] = P;
      eend[sg * nsys + l] = yl;
    }
    __syncthreads();
    if (act) {
      if (sg > 0) {
        double c = 0.0;
        for (int h = 0; h < kSegMax; h += 8) {  // 8 segment ends per round of loads
          double pe[8], ee[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const int j = min(h + k, S - 1);
            pe[k] = pend[j * nb + q];
            ee[k] = eend[j * nsys + l];
          }
#pragma unroll
          for (int k = 0; k < 8; ++k)
            if (h + k < sg) c = fma(pe[k], c, ee[k]);
        }
        double Pk = 1.0;
#pragma unroll
        for (int k = 0; k < kSegReg; ++k) {
          Pk *= bf[k];
          y[k] = fma(Pk, c, y[k]);
        }
      }
      double xl = 0.0, Q = 1.0;
#pragma unroll
      for (int k = kSegReg - 1; k >= 0; --k) {
        if (k < cnt) {
          xl = fma(bb[k], xl, y[k]);
          Q *= bb[k];
        }
        y[k] = xl;
      }
      if (S > 1) {
        if ((l & QS) == 0) pendB[sg * nb + q] = Q;
        eendB[sg * nsys + l] = xl;
      }
    }
    __syncthreads();
    if (act) {
      if (sg < S - 1) {
        double c = 0.0;
        for (int h = kSegMax - 8; h >= 0; h -= 8) {
          double pe[8], ee[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const int j = min(h + k, S - 1);
            pe[k] = pendB[j * nb + q];
            ee[k] = eendB[j * nsys + l];
          }
#pragma unroll
          for (int k = 7; k >= 0; --k)
            if (h + k > sg && h + k < S) c = fma(pe[k], c, ee[k]);
        }
        double Qk = 1.0;
#pragma unroll
        for (int k = kSegReg - 1; k >= 0; --k) {
          if (k < cnt) {
            Qk *= bb[k];
            y[k] = fma(Qk, c, y[k]);
          }
        }
      }
#pragma unroll
      for (int k = 0; k < kSegReg; ++k)
        if (k < cnt) w[(beg + k) * ws + l] = y[k];
    }
  } else {
    // forward sweep, local part
    for (int t = threadIdx.x; t < nsys * S; t += blockDim.x) {
      const int l = t % nsys, sg = t / nsys, q = l >> QS;
      const int beg = sg * len, end = min(na, beg + len);
      double y = 0.0, P = 1.0;
      for (int i0 = beg; i0 < end; i0 += kSepChunk) {
        double v[kSepChunk], pv[kSepChunk], dv[kSepChunk];
  #pragma unroll
        for (int k = 0; k < kSepChunk; ++k) {
          const int i = min(i0 + k, end - 1);
          v[k] = w[i * ws + l];
          pv[k] = id[i * nb + q];
          dv[k] = i > 0 ? T.da[i] : 0.0;
        }
  #pragma unroll
        for (int k = 0; k < kSepChunk; ++k) {
          const double a = v[k] * pv[k], b = -dv[k] * pv[k];
          if (i0 + k < end) {
            y = fma(b, y, a);
            P *= b;
          }
          v[k] = y;
        }
  #pragma unroll
        for (int k = 0; k < kSepChunk; ++k)
          if (i0 + k < end) w[(i0 + k) * ws + l] = v[k];
      }
      if (S > 1) {
        if ((l & QS) == 0) pend[sg * nb + q] = P;
        eend[sg * nsys + l] = y;
      }
    }
    if (S > 1) {
      __syncthreads();
      for (int t = threadIdx.x; t < nsys * S; t += blockDim.x) {
        const int l = t % nsys, sg = t / nsys, q = l >> QS;
        if (sg == 0) continue;
        double c = 0.0;
        for (int s2 = 0; s2 < sg; ++s2) c = fma(pend[s2 * nb + q], c, eend[s2 * nsys + l]);
        const int beg = sg * len, end = min(na, beg + len);
        double P = 1.0;
        for (int i0 = beg; i0 < end; i0 += kSepChunk) {
          double v[kSepChunk], pv[kSepChunk], dv[kSepChunk];
  #pragma unroll
          for (int k = 0; k < kSepChunk; ++k) {
            const int i = min(i0 + k, end - 1);
            v[k] = w[i * ws + l];
            pv[k] = id[i * nb + q];
            dv[k] = T.da[i];
          }
  #pragma unroll
          for (int k = 0; k < kSepChunk; ++k) {
            P *= -dv[k] * pv[k];
            v[k] = fma(P, c, v[k]);
          }
  #pragma unroll
          for (int k = 0; k < kSepChunk; ++k)
            if (i0 + k < end) w[(i0 + k) * ws + l] = v[k];
        }
      }
    }
    __syncthreads();
    // back substitution, local part
    for (int t = threadIdx.x; t < nsys * S; t += blockDim.x) {
      const int l = t % nsys, sg = t / nsys, q = l >> QS;
      const int beg = sg * len, end = min(na, beg + len);
      double x = 0.0, Q = 1.0;
      for (int i1 = end - 1; i1 >= beg; i1 -= kSepChunk) {
        double v[kSepChunk], cv[kSepChunk];
  #pragma unroll
        for (int k = 0; k < kSepChunk; ++k) {
          const int i = max(i1 - k, beg);
          v[k] = w[i * ws + l];
          cv[k] = i < na - 1 ? cp[i * nb + q] : 0.0;
        }
  #pragma unroll
        for (int k = 0; k < kSepChunk; ++k) {
          if (i1 - k >= beg) {
            x = fma(-cv[k], x, v[k]);
            Q *= -cv[k];
          }
          v[k] = x;
        }
  #pragma unroll
        for (int k = 0; k < kSepChunk; ++k)
          if (i1 - k >= beg) w[(i1 - k) * ws + l] = v[k];
      }
      if (S > 1) {
        if ((l & QS) == 0) pend[sg * nb + q] = Q;
        eend[sg * nsys + l] = x;
      }
    }
    if (S > 1) {
      __syncthreads();
      for (int t = threadIdx.x; t < nsys * S; t += blockDim.x) {
        const int l = t % nsys, sg = t / nsys, q = l >> QS;
        if (sg == S - 1) continue;
        double c = 0.0;
        for (int s2 = S - 1; s2 > sg; --s2) c = fma(pend[s2 * nb + q], c, eend[s2 * nsys + l]);
        const int beg = sg * len, end = min(na, beg + len);
        double Q = 1.0;
        for (int i1 = end - 1; i1 >= beg; i1 -= kSepChunk) {
          double v[kSepChunk], cv[kSepChunk];
  #pragma unroll
          for (int k = 0; k < kSepChunk; ++k) {
            const int i = max(i1 - k, beg);
            v[k] = w[i * ws + l];
            cv[k] = cp[i * nb + q];
          }
  #pragma unroll
          for (int k = 0; k < kSepChunk; ++k) {
            Q *= -cv[k];
            v[k] = fma(Q, c, v[k]);
          }
  #pragma unroll
          for (int k = 0; k < kSepChunk; ++k)
            if (i1 - k >= beg) w[(i1 - k) * ws + l] = v[k];
        }
      }
    }
  }
  __syncthreads();
  sep_rows<QS>(w, na, nb, ws, vt);
  __syncthreads();
}

// Byte offsets of the fused cycle's LDS arrays: o[l] u of level l and
// o[K + l] its f (l < cl, K = kMaxLdsLevels), o[2K + l] the tables of level
// l (l <= cl), o[3K] the coarsest u (its f follows), o[3K + 1] the
// exact-line scratch, o[3K + 2] the total.  Plain layout: [coarsest u, f]
// [levels 0..cl-1: u, f] [scratch] [tables].  Aliased layout: [level 0 u]
// [region A] [scratch] [tables], where region A holds level 0's f while
// level 0 is smoothed and [coarsest u, f] [levels 1..cl-1: u, f] between
// the restriction from level 0 and the prolongation to it.
constexpr int kLayoutSlots = kLdsLayoutSlots;
template <typename R>
__host__ __device__ inline void lds_layout(const LdsLevels& LL, int* o) {
  using V = typename Vec<R>::T;
  constexpr int K = kMaxLdsLevels;
  const int cl = LL.n - 1;
  auto al = [](int x) { return (x + 15) & ~15; };
  auto ub = [&](int l) { return (int)sizeof(V) * (LL.L[l].na + 2) * lvl_us(LL.L[l].nb); };
  auto fb = [&](int l) { return (int)sizeof(V) * LL.L[l].na * lvl_fs(LL.L[l].nb); };
  const bool sep = LL.L[cl].sep_v != nullptr;
  const int nac = LL.L[cl].na, nbc = LL.L[cl].nb;
  // coarsest block: [u padded (SOR fallback)] f, then (exact solve) the
  // staged Thomas factors of the level, 2 na nb doubles, and the segment-end
  // scratch of the tridiagonal solves
  const int cbf = al((int)sizeof(double2) * ((sep ? 0 : (nac + 2) * (nbc + 2)) + nac * nbc));
  const int cb = cbf + (sep ? al((int)sizeof(double) * (2 * nac * nbc + 6 * sep_seg_max(nbc) * nbc)) : 0);
  int q = 0;
  if (LL.alias && cl > 0) {
    o[0] = 0;
    const int a = al(ub(0));
    o[K] = a;
    int c = a;
    o[3 * K] = c;
    c = al(c + cb);
    for (int l = 1; l < cl; ++l) {
      o[l] = c;
      c = al(c + ub(l));
      o[K + l] = c;
      c = al(c + fb(l));
    }
    q = al(a + fb(0)) > c ? al(a + fb(0)) : c;
  } else {
    o[3 * K] = 0;
    q = al(cb);
    for (int l = 0; l < cl; ++l) {
      o[l] = q;
      q = al(q + ub(l));
      o[K + l] = q;
      q = al(q + fb(l));
    }
  }
  o[3 * K + 4] = o[3 * K] + cbf;  // staged Thomas factors of the exact coarse solve
  o[3 * K + 1] = q;
  q = al(q + (int)sizeof(R) * LL.scratch);
  o[2 * K + cl] = q;  // coarsest tables (double)
  q = al(q + (int)sizeof(double) * (5 * LL.L[cl].na + 4 * LL.L[cl].nb));
  o[3 * K + 3] = q;   // staged eigenvector tables (V^T, V^-T) of the exact coarse solve
  q = al(q + (sep ? (int)sizeof(double) * 2 * nbc * nbc : 0));
  for (int l = 0; l < cl; ++l) {
    o[2 * K + l] = q;
    q = al(q + (int)sizeof(R) * (5 * LL.L[l].na + 4 * LL.L[l].nb));
  }
  o[3 * K + 2] = q;
}

template <int PMAX, int NT, typename R>
__global__ void __launch_bounds__(NT) k_lds_cycle(const LdsJob* __restrict__ jobs, BatchRef bt, int nu_pre,
                                                       int nu_post, int n_sor, int exact, double rtol, int max_sweeps) {
  using V = typename Vec<R>::T;
  extern __shared__ char smem[];
  __shared__ double redbuf[NT / 64];
  Red red{redbuf};
  const int p = blockIdx.x;
  int e;
  if (!batch_entry(bt, p, e)) return;
  const LdsJob& J = jobs[ent_prob(e)];
  const LdsLevels& LL = J.LL;
  const int slot = ent_slot(e);
  const int m = J.mode ? J.mode[slot] : slot;
  const auto Fg = gbl(static_cast<const V*>(J.f));
  const auto Ug = gbl(static_cast<V*>(J.u));
  const int load_u = J.load_u;
  const int n = LL.n;
  const int cl = n - 1;  // coarsest level (FP64 storage)
  const int alias = LL.alias;
  const LevelDev& LC = LL.L[cl];
  // per-level byte offsets into LDS of u, f and the staged tables (kept in
  // LDS and turned into pointers at each use, so that the pointers stay
  // known as LDS addresses and no per-thread array is indexed dynamically)
  __shared__ int s_off[kLayoutSlots];
  for (int t = threadIdx.x; t < kLayoutSlots; t += blockDim.x) s_off[t] = J.off[t];  // laid out by the host
  __syncthreads();
  // coarsest arrays: f (and, for the SOR fallback, the padded u before it)
  const bool sep = LC.sep_v != nullptr;
  double2* uC = reinterpret_cast<double2*>(smem + s_off[3 * kMaxLdsLevels]);
  double2* fC = sep ? uC : uC + (LC.na + 2) * (LC.nb + 2);
  auto Ul = [&](int l) { return reinterpret_cast<V*>(smem + s_off[l]); };
  auto Fl = [&](int l) { return reinterpret_cast<V*>(smem + s_off[kMaxLdsLevels + l]); };
  auto Tl = [&](int l) {
    return tab_at<R>(reinterpret_cast<R*>(smem + s_off[2 * kMaxLdsLevels + l]), LL.L[l].na, LL.L[l].nb);
  };
  R* cp = reinterpret_cast<R*>(smem + s_off[3 * kMaxLdsLevels + 1]);
  Tab<double> tabC = stage_tab<double>(LC, m, reinterpret_cast<double*>(smem + s_off[2 * kMaxLdsLevels + cl]));
  double* sepV = reinterpret_cast<double*>(smem + s_off[3 * kMaxLdsLevels + 3]);
  double* sepF = reinterpret_cast<double*>(smem + s_off[3 * kMaxLdsLevels + 4]);
  // A kernel whose only level is the coarsest stages the Thomas factors and
  // f together with the eigenvector tables (one round of memory latency);
  // otherwise the factors share LDS with the finer levels and are staged by
  // the coarse solve itself.
  const bool pre = sep && n == 1;
  if (sep) {
    const int nn = LC.nb * LC.nb, nf = pre ? LC.na * LC.nb : 0;
    const auto gv = gbl(LC.sep_v + (size_t)m * nn), gvi = gbl(LC.sep_vi + (size_t)m * nn);
    const auto gcp = gbl(LC.sep_cp + (size_t)m * LC.na * LC.nb), gid = gbl(LC.sep_id + (size_t)m * LC.na * LC.nb);
    const size_t off = (size_t)slot * LC.na * LC.nb;
    // even sizes (the usual case): pairs of entries per 16-byte load (the
    // tables and planes start on 16-byte boundaries); else one per load
    const int nn2 = nn / 2, nf2 = nf / 2;
    const bool pairs = (nn & 1) == 0 && (nf & 1) == 0;
#pragma unroll 2
    for (int t = threadIdx.x; pairs && t < max(nn2, nf2); t += blockDim.x) {
      double2 v0 = make_double2(0.0, 0.0), v1 = v0, c0 = v0, c1 = v0;
      V fa = mkv<R>(0, 0), fb = fa;
      if (t < nn2) {
        v0 = gbl(reinterpret_cast<const double2*>(LC.sep_v + (size_t)m * nn))[t];
        v1 = gbl(reinterpret_cast<const double2*>(LC.sep_vi + (size_t)m * nn))[t];
      }
      if (t < nf2) {
        c0 = gbl(reinterpret_cast<const double2*>(LC.sep_cp + (size_t)m * LC.na * LC.nb))[t];
        c1 = gbl(reinterpret_cast<const double2*>(LC.sep_id + (size_t)m * LC.na * LC.nb))[t];
        if constexpr (sizeof(V) == 8) {
          const float4 f4 = gbl(reinterpret_cast<const float4*>(static_cast<const V*>(J.f) + off))[t];
          fa = mkv<R>(f4.x, f4.y);
          fb = mkv<R>(f4.z, f4.w);
        } else {
          fa = Fg[off + 2 * t];
          fb = Fg[off + 2 * t + 1];
        }
      }
      if (t < nn2) {
        sepV[2 * t] = v0.x;
        sepV[2 * t + 1] = v0.y;
        sepV[nn + 2 * t] = v1.x;
        sepV[nn + 2 * t + 1] = v1.y;
      }
      if (t < nf2) {
        sepF[2 * t] = c0.x;
        sepF[2 * t + 1] = c0.y;
        sepF[nf + 2 * t] = c1.x;
        sepF[nf + 2 * t + 1] = c1.y;
        fC[2 * t] = make_double2(fa.x, fa.y);
        fC[2 * t + 1] = make_double2(fb.x, fb.y);
      }
    }
#pragma unroll 4
    for (int t = threadIdx.x; !pairs && t < max(nn, nf); t += blockDim.x) {
      double v0 = 0.0, v1 = 0.0, c0 = 0.0, c1 = 0.0;
      V fv = mkv<R>(0, 0);
      if (t < nn) {
        v0 = gv[t];
        v1 = gvi[t];
      }
      if (t < nf) {
        c0 = gcp[t];
        c1 = gid[t];
        fv = Fg[off + t];
      }
      if (t < nn) {
        sepV[t] = v0;
        sepV[nn + t] = v1;
      }
      if (t < nf) {
        sepF[t] = c0;
        sepF[nf + t] = c1;
        fC[t] = make_double2(fv.x, fv.y);
      }
    }
  }
  for (int l = 0; l < cl; ++l) (void)stage_tab<R>(LL.L[l], m, reinterpret_cast<R*>(smem + s_off[2 * kMaxLdsLevels + l]));
  // level 0 of the fused range: load f (and u for a full in-LDS cycle)
  {
    const LevelDev& L0 = LL.L[0];
    const int na = L0.na, nb = L0.nb;
    const size_t off = (size_t)slot * na * nb;
    if (n > 1) {
      const int nc = lvl_us(nb), fs = lvl_fs(nb);
#pragma unroll 4
      for (int t = threadIdx.x; t < (na + 2) * nc; t += blockDim.x) {
        const int i = t / nc - 1, j = t % nc - 1;
        V v = mkv<R>(0, 0);
        if (load_u && i >= 0 && i < na && j >= 0 && j < nb) v = Ug[off + (size_t)i * nb + j];
        Ul(0)[t] = v;
      }
#pragma unroll 4
      for (int t = threadIdx.x; t < na * nb; t += blockDim.x) {
        const int i = t / nb, j = t - i * nb;
        Fl(0)[i * fs + j] = Fg[off + t];
      }
    } else if (!pre) {
#pragma unroll 4
      for (int t = threadIdx.x; t < na * nb; t += blockDim.x) {
        const V v = Fg[off + t];
        fC[t] = make_double2(v.x, v.y);
      }
    }
  }
  __syncthreads();
  // descend
  for (int l = 0; l < cl; ++l) {
    const LevelDev& L = LL.L[l];
    const LevelDev& C = LL.L[l + 1];
    const Tab<R> T = Tl(l);
    V* ul = Ul(l);
    const V* fl = Fl(l);
    for (int k = 0; k < nu_pre; ++k) smooth_step<PMAX, R>(L, T, ul, fl, n_sor, exact, cp);
    // coarse u is cleared over its padded extent (row stride ncc), coarse f
    // is stored with row stride fcs
    const int ncc = l + 1 == cl ? C.nb + 2 : lvl_us(C.nb);
    const int fcs = l + 1 == cl ? C.nb : lvl_fs(C.nb);
    // coarse right-hand side = area-weighted restriction of the residual
    auto restrict_at = [&](int t) {
      const int I = t / C.nb, J = t - I * C.nb;
      R ax = 0, ay = 0;
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
          const R w = (R)gbl(L.rwa)[2 * I + a] * (R)gbl(L.rwb)[2 * J + b];
          const V r = resid_lds<R>(L, T, ul, fl, 2 * I + a, 2 * J + b, lvl_us(L.nb), lvl_fs(L.nb));
          ax = fma(w, r.x, ax);
          ay = fma(w, r.y, ay);
        }
      return mkv<R>(ax, ay);
    };
    auto put_f = [&](int t, V v) {
      const int I = t / C.nb, J = t - I * C.nb;
      if (l + 1 == cl) fC[t] = make_double2(v.x, v.y);
      else Fl(l + 1)[I * fcs + J] = v;
    };
    if (alias && l == 0) {
      // the coarse arrays overlay this level's f: restrict into registers
      // (at most kAliasCells per thread), then clear and store
      V acc[kAliasCells];
#pragma unroll
      for (int k = 0; k < kAliasCells; ++k) {
        const int t = threadIdx.x + k * blockDim.x;
        acc[k] = t < C.na * C.nb ? restrict_at(t) : mkv<R>(0, 0);
      }
      __syncthreads();
      if (l + 1 < cl)
        for (int t = threadIdx.x; t < (C.na + 2) * ncc; t += blockDim.x) Ul(l + 1)[t] = mkv<R>(0, 0);
#pragma unroll
      for (int k = 0; k < kAliasCells; ++k) {
        const int t = threadIdx.x + k * blockDim.x;
        if (t < C.na * C.nb) put_f(t, acc[k]);
      }
    } else {
      if (l + 1 < cl)
        for (int t = threadIdx.x; t < (C.na + 2) * ncc; t += blockDim.x) Ul(l + 1)[t] = mkv<R>(0, 0);
      for (int t = threadIdx.x; t < C.na * C.nb; t += blockDim.x) put_f(t, restrict_at(t));
    }
    __syncthreads();
  }
  // coarsest level in FP64, solved exactly by fast diagonalisation when its
  // factors exist (the solution replaces f in place), otherwise by red-black
  // SOR from zero until the residual 2-norm dropped by rtol (Sec. 3.3)
  if (sep) {
    coarse_separable<1>(LC, tabC, m, reinterpret_cast<double*>(fC), 2 * LC.nb, sepV, sepF, pre);
  } else {
    const LevelDev& L = LC;
    const Tab<double>& T = tabC;
    const int na = L.na, nb = L.nb, nc = nb + 2;
    for (int t = threadIdx.x; t < (na + 2) * nc; t += blockDim.x) uC[t] = make_double2(0.0, 0.0);
    __syncthreads();
    double f2 = 0.0;
    for (int t = threadIdx.x; t < na * nb; t += blockDim.x) f2 += fC[t].x * fC[t].x + fC[t].y * fC[t].y;
    f2 = red.sum(f2);
    const double w = gbl(L.wc)[m];
    if (f2 > 0.0) {
      for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        for (int colour = 0; colour < 2; ++colour) {
          for (int t = threadIdx.x; t < na * nb; t += blockDim.x) {
            const int i = t / nb, j = t - i * nb;
            if (((i + j) & 1) != colour) continue;
            const int qq = (i + 1) * nc + (j + 1);
            const double Rr = T.Rr[i];
            const double c = T.Ca[i] + Rr * T.Cb[j];
            const double a1 = T.ua[i], a2 = T.da[i], b1 = Rr * T.ub[j], b2 = Rr * T.db[j];
            const double2 un = uC[qq + nc], us = uC[qq - nc], ue = uC[qq + 1], uw = uC[qq - 1];
            const double2 fv = fC[t];
            const double tx = (fv.x - (a1 * un.x + a2 * us.x + b1 * ue.x + b2 * uw.x)) / c;
            const double ty = (fv.y - (a1 * un.y + a2 * us.y + b1 * ue.y + b2 * uw.y)) / c;
            const double2 old = uC[qq];
            uC[qq] = make_double2(old.x + w * (tx - old.x), old.y + w * (ty - old.y));
          }
          __syncthreads();
        }
        double r2 = 0.0;
        for (int t = threadIdx.x; t < na * nb; t += blockDim.x) {
          const int i = t / nb, j = t - i * nb;
          const double2 r = resid_lds<double>(L, T, uC, fC, i, j, nb + 2, nb);
          r2 += r.x * r.x + r.y * r.y;
        }
        r2 = red.sum(r2);
        if (r2 <= rtol * rtol * f2) break;
      }
    }
    __syncthreads();
  }
  // ascend
  for (int l = cl - 1; l >= 0; --l) {
    const LevelDev& L = LL.L[l];
    const LevelDev& C = LL.L[l + 1];
    const int nb = L.nb, nc = lvl_us(nb), ncc = l + 1 == cl ? C.nb + 2 : lvl_us(C.nb);
    const int par = m & 1;
    const Tab<R> T = Tl(l);
    V* ul = Ul(l);
    const V* fl = Fl(l);
#pragma unroll 4
    for (int t = threadIdx.x; t < L.na * nb; t += blockDim.x) {
      const int i = t / nb, j = t - i * nb;
      const int a0 = gbl(L.pa_i0)[i], a1 = gbl(L.pa_i1)[i];
      const int b0 = gbl(L.pb_i0)[par * nb + j], b1 = gbl(L.pb_i1)[par * nb + j];
      const R wa0 = (R)gbl(L.pa_w0)[i], wa1 = (R)gbl(L.pa_w1)[i];
      const R wb0 = (R)gbl(L.pb_w0)[par * nb + j], wb1 = (R)gbl(L.pb_w1)[par * nb + j];
      R e00x, e00y, e01x, e01y, e10x, e10y, e11x, e11y;
      if (l + 1 == cl) {
        // the coarsest solution: padded u (SOR) or, unpadded, in f (exact
        // solve; ghost neighbours read as zero)
        auto cv = [&](int ia, int jb) {
          if (!sep) return uC[(ia + 1) * ncc + jb + 1];
          return (ia >= 0 && ia < C.na && jb >= 0 && jb < C.nb) ? fC[ia * C.nb + jb] : make_double2(0.0, 0.0);
        };
        const double2 a = cv(a0, b0), b = cv(a0, b1), c = cv(a1, b0), d = cv(a1, b1);
        e00x = (R)a.x; e00y = (R)a.y; e01x = (R)b.x; e01y = (R)b.y;
        e10x = (R)c.x; e10y = (R)c.y; e11x = (R)d.x; e11y = (R)d.y;
      } else {
        const V* uc = Ul(l + 1);
        const V a = uc[(a0 + 1) * ncc + b0 + 1], b = uc[(a0 + 1) * ncc + b1 + 1];
        const V c = uc[(a1 + 1) * ncc + b0 + 1], d = uc[(a1 + 1) * ncc + b1 + 1];
        e00x = a.x; e00y = a.y; e01x = b.x; e01y = b.y; e10x = c.x; e10y = c.y; e11x = d.x; e11y = d.y;
      }
      R ex = 0, ey = 0;
      ex = fma(wa0 * wb0, e00x, ex); ey = fma(wa0 * wb0, e00y, ey);
      ex = fma(wa0 * wb1, e01x, ex); ey = fma(wa0 * wb1, e01y, ey);
      ex = fma(wa1 * wb0, e10x, ex); ey = fma(wa1 * wb0, e10y, ey);
      ex = fma(wa1 * wb1, e11x, ex); ey = fma(wa1 * wb1, e11y, ey);
      const int qq = (i + 1) * nc + (j + 1);
      ul[qq] = mkv<R>(ul[qq].x + ex, ul[qq].y + ey);
    }
    __syncthreads();
    if (alias && l == 0) {
      // the coarse levels are done with region A: level 0's f again
      const size_t off = (size_t)slot * L.na * nb;
      const int fs = lvl_fs(nb);
#pragma unroll 4
      for (int t = threadIdx.x; t < L.na * nb; t += blockDim.x) {
        const int i = t / nb, j = t - i * nb;
        Fl(0)[i * fs + j] = Fg[off + t];
      }
      __syncthreads();
    }
    for (int k = 0; k < nu_post; ++k) smooth_step<PMAX, R>(L, T, ul, fl, n_sor, exact, cp);
  }
  {
    const LevelDev& L0 = LL.L[0];
    const int na = L0.na, nb = L0.nb, nc = n > 1 ? lvl_us(nb) : nb + 2;
    const size_t off = (size_t)slot * na * nb;
    for (int t = threadIdx.x; t < na * nb; t += blockDim.x) {
      const int i = t / nb, j = t - i * nb;
      if (n > 1) {
        Ug[off + t] = Ul(0)[(i + 1) * nc + (j + 1)];
      } else {
        const double2 v = sep ? fC[t] : uC[(i + 1) * nc + (j + 1)];
        Ug[off + t] = mkv<R>((R)v.x, (R)v.y);
      }
    }
  }
}

// Exact coarsest solve of planes whose only level in the launch is the
// coarsest, with separable factors: the operator is real, so the real and the
// imaginary part of a plane are independent problems, and each gets a block
// of its own (twice the blocks of one per plane, half the work per block).
// The component sits in LDS as a real plane of row stride split_ws(nb)
// doubles, 4 more than a multiple of 32, which spreads the 16 rows a matrix
// core operand reads over the LDS banks.  The arithmetic per element is that
// of the complex path, so both give the same bits.
__host__ __device__ inline int split_ws(int nb) { return nb + ((4 - nb % 32) + 32) % 32; }

// LDS layout in doubles: o[0] eigenvector tables (V^T, V^-T), o[1] Thomas
// factors and segment-end scratch, o[2] the plane, o[3] the radial table da
// of the sweeps, o[4] the total.
__host__ __device__ inline void split_layout(int na, int nb, int* o) {
  auto al = [](int x) { return (x + 1) & ~1; };
  const int S = sep_seg_max(nb);
  o[0] = 0;
  o[1] = al(2 * nb * nb);
  o[2] = o[1] + al(2 * na * nb + 4 * S * nb);
  o[3] = o[2] + al(na * split_ws(nb));
  o[4] = o[3] + al(na);
}

constexpr int kSplitThreads = 256;  // >= nb sep_seg_max(nb) for every nb

template <typename R>
__global__ void __launch_bounds__(kSplitThreads) k_coarse_split(const LdsJob* __restrict__ jobs, BatchRef bt) {
  using V = typename Vec<R>::T;
  extern __shared__ char smem[];
  const int p = blockIdx.x, comp = blockIdx.y;
  int e;
  if (!batch_entry(bt, p, e)) return;
  // the job's fields, read in one round before the mode lookup branches
  const LdsJob& J = jobs[ent_prob(e)];
  const LevelDev LC = J.LL.L[0];
  void* const ju = J.u;
  const void* const jf = J.f;
  const int* const jmode = J.mode;
  for (const void* v : {(const void*)jmode, (const void*)ju, jf, (const void*)LC.sep_v, (const void*)LC.sep_vi,
                        (const void*)LC.sep_cp, (const void*)LC.sep_id, (const void*)LC.da})
    pin_scalar(v);
  pin_scalar(LC.na);
  pin_scalar(LC.nb);
  const int slot = ent_slot(e);
  const int m = jmode ? jmode[slot] : slot;
  const int na = LC.na, nb = LC.nb, nn = na * nb, nv = nb * nb, ws = split_ws(nb);
  int o[5];
  split_layout(na, nb, o);
  double* D = reinterpret_cast<double*>(smem);
  double* sepV = D + o[0];
  double* sepF = D + o[1];
  double* X = D + o[2];
  const size_t off = (size_t)slot * nn;
  const V* fv = static_cast<const V*>(jf) + off;
  // stage the eigenvector tables, the Thomas factors, this component of f
  // and the sweeps' one 1D table (da), all loads in flight together; pairs
  // of entries per 16-byte load when the sizes are even (tables and planes
  // start on 16-byte boundaries)
  double* const da = D + o[3];
  double da0 = 0.0;  // da of row threadIdx.x (clamped), loaded with the first batch
  const bool pairs = (nb & 1) == 0;
  const int nv2 = nv / 2, nn2 = nn / 2;
  const auto gv2 = gbl(reinterpret_cast<const double2*>(LC.sep_v + (size_t)m * nv));
  const auto gvi2 = gbl(reinterpret_cast<const double2*>(LC.sep_vi + (size_t)m * nv));
  const auto gcp2 = gbl(reinterpret_cast<const double2*>(LC.sep_cp + (size_t)m * nn));
  const auto gid2 = gbl(reinterpret_cast<const double2*>(LC.sep_id + (size_t)m * nn));
  // one pair position of every array into LDS (component comp of f)
  auto put = [&](int t, double2 v0, double2 v1, double2 c0, double2 c1, double fa, double fb) {
    if (t < nv2) {
      sepV[2 * t] = v0.x;
      sepV[2 * t + 1] = v0.y;
      sepV[nv + 2 * t] = v1.x;
      sepV[nv + 2 * t + 1] = v1.y;
    }
    if (t < nn2) {
      sepF[2 * t] = c0.x;
      sepF[2 * t + 1] = c0.y;
      sepF[nn + 2 * t] = c1.x;
      sepF[nn + 2 * t + 1] = c1.y;
      const int i = 2 * t / nb, j = 2 * t - i * nb;  // nb even: both cells in row i
      X[i * ws + j] = fa;
      X[i * ws + j + 1] = fb;
    }
  };
  auto f_pair = [&](int t, double& fa, double& fb) {
    if constexpr (sizeof(V) == 8) {
      const float4 f4 = gbl(reinterpret_cast<const float4*>(fv))[t];
      fa = comp ? f4.y : f4.x;
      fb = comp ? f4.w : f4.z;
    } else {
      const V a = gbl(fv)[2 * t], b = gbl(fv)[2 * t + 1];
      fa = comp ? a.y : a.x;
      fb = comp ? b.y : b.x;
    }
  };
  if (pairs) {
    // the first kStageBatch positions per thread: every load issued before
    // any store (indices clamped into range, so no load sits behind a
    // branch), then the stores; larger planes continue in a strided loop
    constexpr int kStageBatch = 4;
    double2 v0[kStageBatch], v1[kStageBatch], c0[kStageBatch], c1[kStageBatch];
    double fa[kStageBatch], fb[kStageBatch];
#pragma unroll
    for (int k = 0; k < kStageBatch; ++k) {
      const int t = threadIdx.x + k * (int)blockDim.x;
      const int tv = min(t, nv2 - 1), tn = min(t, nn2 - 1);
      if (k == 0) da0 = gbl(LC.da)[min((int)threadIdx.x, na - 1)];
      v0[k] = gv2[tv];
      v1[k] = gvi2[tv];
      c0[k] = gcp2[tn];
      c1[k] = gid2[tn];
      f_pair(tn, fa[k], fb[k]);
    }
#pragma unroll
    for (int k = 0; k < kStageBatch; ++k)
      put(threadIdx.x + k * (int)blockDim.x, v0[k], v1[k], c0[k], c1[k], fa[k], fb[k]);
    for (int t = threadIdx.x + kStageBatch * (int)blockDim.x; t < max(nv2, nn2); t += blockDim.x) {
      double2 a0 = make_double2(0.0, 0.0), a1 = a0, b0 = a0, b1 = a0;
      double ga = 0.0, gb = 0.0;
      if (t < nv2) {
        a0 = gv2[t];
        a1 = gvi2[t];
      }
      if (t < nn2) {
        b0 = gcp2[t];
        b1 = gid2[t];
        f_pair(t, ga, gb);
      }
      put(t, a0, a1, b0, b1, ga, gb);
    }
  }
  if (!pairs) da0 = gbl(LC.da)[min((int)threadIdx.x, na - 1)];
#pragma unroll 4
  for (int t = threadIdx.x; !pairs && t < max(nv, nn); t += blockDim.x) {
    double v0 = 0.0, v1 = 0.0, c0 = 0.0, c1 = 0.0, fa = 0.0;
    if (t < nv) {
      v0 = gbl(LC.sep_v + (size_t)m * nv)[t];
      v1 = gbl(LC.sep_vi + (size_t)m * nv)[t];
    }
    if (t < nn) {
      c0 = gbl(LC.sep_cp + (size_t)m * nn)[t];
      c1 = gbl(LC.sep_id + (size_t)m * nn)[t];
      const V a = gbl(fv)[t];
      fa = comp ? a.y : a.x;
    }
    if (t < nv) {
      sepV[t] = v0;
      sepV[nv + t] = v1;
    }
    if (t < nn) {
      sepF[t] = c0;
      sepF[nn + t] = c1;
      const int i = t / nb;
      X[i * ws + (t - i * nb)] = fa;
    }
  }
  if (threadIdx.x < na) da[threadIdx.x] = da0;
  for (int i = threadIdx.x + blockDim.x; i < na; i += blockDim.x) da[i] = gbl(LC.da)[i];
  Tab<double> T{};
  T.da = da;  // the only table the exact solve reads
  __syncthreads();
  coarse_separable<0>(LC, T, m, X, ws, sepV, sepF, true);
  R* ug = reinterpret_cast<R*>(static_cast<V*>(ju) + off) + comp;
#pragma unroll 4
  for (int t = threadIdx.x; t < nn; t += blockDim.x) {
    const int i = t / nb;
    ug[2 * t] = (R)X[i * ws + (t - i * nb)];
  }
}

template <typename R>
size_t cycle_bytes(const LdsLevels& LL) {
  int o[kLayoutSlots];
  lds_layout<R>(LL, o);
  return (size_t)o[3 * kMaxLdsLevels + 2];
}

int cycle_threads(const LdsLevels& LL) {
  // enough waves that each takes about one line group per colour on the
  // first fused level; few threads keep the barriers of small levels cheap
  const int cells = LL.L[0].na * LL.L[0].nb;
  return cells >= 8192 ? 1024 : (cells >= 2048 ? 512 : (cells >= 512 ? 256 : 64));
}

}  // namespace

namespace smgk {

int lds_cycle_scratch(const LdsLevels& LL, bool exact) {
  size_t scratch = 0;
  if (exact)
    for (int l = 0; l + 1 < LL.n; ++l) {
      const size_t a = (size_t)((LL.L[l].nb + 1) / 2) * LL.L[l].na;
      const size_t b = (size_t)((LL.L[l].na + 1) / 2) * LL.L[l].nb;
      scratch = scratch > a ? scratch : a;
      scratch = scratch > b ? scratch : b;
    }
  return (int)((scratch + 1) / 2 * 2);  // even: keeps the FP64 tables that follow 8-byte aligned
}

void lds_cycle_layout(const LdsLevels& LL, bool fp32, int* off) {
  if (fp32) lds_layout<float>(LL, off);
  else lds_layout<double>(LL, off);
}

size_t lds_cycle_bytes(const LdsLevels& LL, bool fp32) {
  return fp32 ? cycle_bytes<float>(LL) : cycle_bytes<double>(LL);
}

bool lds_cycle_alias_ok(const LdsLevels& LL) {
  // every launch has at least min(cycle_threads, 512) threads
  return LL.n > 1 && LL.L[1].na * LL.L[1].nb <= kAliasCells * std::min(cycle_threads(LL), 512);
}

int lds_cycle_threads(const LdsLevels& LL) { return cycle_threads(LL); }

hipError_t mg_lds_cycle(const LdsJob* jobs, const LdsJob* hj, int n_prob, const BatchRef& b, int nu_pre, int nu_post,
                        int n_sor, bool exact, bool fp32, double rtol, int max_sweeps, hipStream_t st) {
  if (!b.cap) return hipSuccess;
  // every plane's only level the separable coarsest: one block per component
  bool split = true;
  size_t slds = 0;
  for (int q = 0; q < n_prob && split; ++q) {
    const LdsLevels& LL = hj[q].LL;
    split = LL.n == 1 && LL.L[0].sep_v != nullptr && LL.L[0].nb <= 16 * kSepMaxTiles;
    if (split) {
      int o[5];
      split_layout(LL.L[0].na, LL.L[0].nb, o);
      slds = std::max(slds, sizeof(double) * (size_t)o[4]);
    }
  }
  if (split && slds <= lds_limit() - 1024) {
    const dim3 grid(b.cap, 2);
    if (fp32) hipLaunchKernelGGL(k_coarse_split<float>, grid, dim3(kSplitThreads), slds, st, jobs, b);
    else hipLaunchKernelGGL(k_coarse_split<double>, grid, dim3(kSplitThreads), slds, st, jobs, b);
    return hipGetLastError();
  }
  size_t lds = 0;
  int threads = 64;
  for (int q = 0; q < n_prob; ++q) {
    lds = std::max(lds, lds_cycle_bytes(hj[q].LL, fp32));
    threads = std::max(threads, cycle_threads(hj[q].LL));
  }
  if (lds > lds_limit() - 1024) return hipErrorInvalidConfiguration;
  int pmax = 2;  // points per lane the longest relaxed line needs
  for (int q = 0; q < n_prob; ++q) {
    for (int l = 0; l + 1 < hj[q].LL.n; ++l) {
      if (hj[q].LL.L[l].na > kRelaxMaxPoints || hj[q].LL.L[l].nb > kRelaxMaxPoints) return hipErrorInvalidConfiguration;
      pmax = std::max(pmax, relax_points_per_lane(std::max(hj[q].LL.L[l].na, hj[q].LL.L[l].nb)));
    }
    if (hj[q].LL.alias && !lds_cycle_alias_ok(hj[q].LL)) return hipErrorInvalidConfiguration;
  }
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(b.cap), dim3(threads), lds, st, jobs, b, nu_pre, nu_post, n_sor, exact ? 1 : 0, rtol,
                       max_sweeps);
  };
  // 1024-thread blocks exist for the FP32 short-line variant only (the
  // others would spill at 128 registers per lane)
  if (!fp32 || pmax > 2) threads = std::min(threads, 512);
  for (int q = 0; q < n_prob; ++q)
    if (hj[q].LL.alias && hj[q].LL.L[1].na * hj[q].LL.L[1].nb > kAliasCells * threads) return hipErrorInvalidConfiguration;
  const bool big = threads > 512;
  if (fp32) {
    if (pmax <= 2) big ? go(k_lds_cycle<2, 1024, float>) : go(k_lds_cycle<2, 512, float>);
    else if (pmax <= 4) go(k_lds_cycle<4, 512, float>);
    else if (pmax <= 8) go(k_lds_cycle<8, 512, float>);
    else go(k_lds_cycle<16, 512, float>);
  } else {
    if (pmax <= 2) go(k_lds_cycle<2, 512, double>);
    else if (pmax <= 4) go(k_lds_cycle<4, 512, double>);
    else if (pmax <= 8) go(k_lds_cycle<8, 512, double>);
    else go(k_lds_cycle<16, 512, double>);
  }
  return hipGetLastError();
}

}  // namespace smgk
