// The coarse end of the V-cycle in one launch: every level whose plane fits
// in LDS (from level `first` down to the coarsest) is processed by one block
// per plane -- pre-smoothing, residual restriction, the coarsest red-black
// SOR (Sec. 3.3), prolongation and post-smoothing -- without touching global
// memory between levels.  The arithmetic is that of the per-level kernels in
// mg.hip (same colour order, same transfer weights, same stopping rule of
// the coarsest solve); only the memory traffic and the launch count differ.
// Templated on the real type R of the smoothing levels; the coarsest level
// is always solved in FP64 (the mixed form keeps the coarsest solve in FP64).
#include <algorithm>

#include "smg_internal.h"
#include "vec.h"

namespace {

constexpr int kThreads = 512;  // most threads of a fused-cycle block

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
    t[i] = (R)L.ua[i];
    t[na + i] = (R)L.da[i];
    t[2 * na + i] = (R)L.Rr[i];
    t[3 * na + i] = (R)L.Ca[(size_t)m * na + i];
    t[4 * na + i] = (R)L.wb[(size_t)m * na + i];
  }
  R* c = buf + 5 * na;
  for (int j = threadIdx.x; j < nb; j += blockDim.x) {
    c[j] = (R)L.ub[j];
    c[nb + j] = (R)L.db[j];
    c[2 * nb + j] = (R)L.Cb[(size_t)m * nb + j];
    c[3 * nb + j] = (R)L.wr[(size_t)m * nb + j];
  }
  return tab_at<R>(buf, na, nb);
}

// Ordering of LDS accesses between the even-odd passes of one line: every
// line is relaxed by a single wave, whose LDS operations complete in issue
// order, so only the compiler must keep the passes apart.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One zebra phase in direction DIR (0: radial lines, fixed j, points along
// i; 1: polar lines, fixed i, points along j): the lines of colour 0, then
// those of colour 1, each line relaxed by n_sor even-odd SOR passes.  A
// wave takes G lines at a time (lane -> line g, point index k of the
// current parity), keeps the stencil coefficients of its two cells (one per
// parity) in registers, and needs no block barrier between the passes of a
// line; one barrier separates the colours.
// u: padded (na+2) x (nb+2) plane, f: na x nb.
template <int DIR, typename R>
__device__ __forceinline__ void sor_phase(const LevelDev& L, const Tab<R>& T, typename Vec<R>::T* u, const typename Vec<R>::T* f,
                          int n_sor) {
  using V = typename Vec<R>::T;
  const int na = L.na, nb = L.nb, nc = nb + 2;
  const int npts = DIR == 0 ? na : nb;
  const int nlines = DIR == 0 ? nb : na;
  const int half = (npts + 1) / 2;                 // points of parity 0
  const int G = half >= 64 ? 1 : 64 / half;        // lines per wave step
  const int cpl = (half + 63) / 64;                // cells per lane and parity
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
  const int g = G > 1 ? lane / half : 0, k0 = G > 1 ? lane - g * half : lane;
  for (int lc = 0; lc < 2; ++lc) {
    const int nlc = (nlines - lc + 1) / 2;          // lines of this colour
    for (int base = wave * G; base < nlc; base += nwave * G) {
      const int li = base + g;                     // this lane's line (colour index)
      const bool lane_ok = (G == 1 || g < G) && li < nlc;
      const int line = lc + 2 * li;
      if (cpl > 1) {
        // lines longer than 128 points: each pass sweeps the lane's cells of
        // that parity, coefficients read as needed
        for (int it = 0; it < n_sor; ++it) {
          for (int pc = 0; pc < 2; ++pc) {
            for (int c = 0; c < cpl && lane_ok; ++c) {
              const int pt = pc + 2 * (k0 + 64 * c);
              if (pt >= npts) break;
              const int i = DIR == 1 ? line : pt, j = DIR == 1 ? pt : line;
              const int qq = (i + 1) * nc + (j + 1);
              const R Rr = T.Rr[i];
              const R cv = T.Ca[i] + Rr * T.Cb[j];
              const R wv = DIR == 1 ? T.wb[i] : T.wr[j];
              const R ua = T.ua[i], da = T.da[i], ub = Rr * T.ub[j], db = Rr * T.db[j];
              const V un = u[qq + nc], us = u[qq - nc], ue = u[qq + 1], uw = u[qq - 1];
              const V fq = f[i * nb + j];
              const R sx = ua * un.x + da * us.x + ub * ue.x + db * uw.x;
              const R sy = ua * un.y + da * us.y + ub * ue.y + db * uw.y;
              const V old = u[qq];
              const R tx = (fq.x - sx) / cv, ty = (fq.y - sy) / cv;
              u[qq] = mkv<R>(old.x + wv * (tx - old.x), old.y + wv * (ty - old.y));
            }
            wave_sync();
          }
        }
        continue;
      }
      {
        const int k = k0;
        // the lane's cell of each parity and its coefficients
        int q[2];
        R cc[2], w[2], a1[2], a2[2], b1[2], b2[2];
        V fv[2];
        bool ok[2];
        for (int pc = 0; pc < 2; ++pc) {
          const int pt = pc + 2 * k;
          ok[pc] = lane_ok && pt < npts;
          const int i = DIR == 1 ? line : pt, j = DIR == 1 ? pt : line;
          q[pc] = (i + 1) * nc + (j + 1);
          if (ok[pc]) {
            const R Rr = T.Rr[i];
            cc[pc] = T.Ca[i] + Rr * T.Cb[j];
            w[pc] = DIR == 1 ? T.wb[i] : T.wr[j];
            a1[pc] = T.ua[i];
            a2[pc] = T.da[i];
            b1[pc] = Rr * T.ub[j];
            b2[pc] = Rr * T.db[j];
            fv[pc] = f[i * nb + j];
          }
        }
        for (int it = 0; it < n_sor; ++it) {
          for (int pc = 0; pc < 2; ++pc) {
            if (ok[pc]) {
              const int qq = q[pc];
              const V un = u[qq + nc], us = u[qq - nc], ue = u[qq + 1], uw = u[qq - 1];
              const R sx = a1[pc] * un.x + a2[pc] * us.x + b1[pc] * ue.x + b2[pc] * uw.x;
              const R sy = a1[pc] * un.y + a2[pc] * us.y + b1[pc] * ue.y + b2[pc] * uw.y;
              const V old = u[qq];
              const R tx = (fv[pc].x - sx) / cc[pc], ty = (fv[pc].y - sy) / cc[pc];
              u[qq] = mkv<R>(old.x + w[pc] * (tx - old.x), old.y + w[pc] * (ty - old.y));
            }
            wave_sync();
          }
        }
      }
    }
    __syncthreads();
  }
}

template <int DIR, typename R>
__device__ __forceinline__ void exact_phase(const LevelDev& L, const Tab<R>& T, typename Vec<R>::T* u, const typename Vec<R>::T* f,
                            R* cp) {
  using V = typename Vec<R>::T;
  const int na = L.na, nb = L.nb, nc = nb + 2;
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
        const V fv = f[i * nb + j];
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

template <typename R>
__device__ __forceinline__ void smooth_step(const LevelDev& L, const Tab<R>& T, typename Vec<R>::T* u, const typename Vec<R>::T* f,
                            int n_sor, bool exact, R* cp) {
  if (exact) {
    exact_phase<0, R>(L, T, u, f, cp);
    exact_phase<1, R>(L, T, u, f, cp);
  } else {
    sor_phase<0, R>(L, T, u, f, n_sor);
    sor_phase<1, R>(L, T, u, f, n_sor);
  }
}

template <typename R>
__device__ __forceinline__ typename Vec<R>::T resid_lds(const LevelDev& L, const Tab<R>& T, const typename Vec<R>::T* u,
                                                        const typename Vec<R>::T* f, int i, int j) {
  const int nb = L.nb, nc = nb + 2;
  const int q = (i + 1) * nc + (j + 1);
  const R Rr = T.Rr[i];
  const R c = T.Ca[i] + Rr * T.Cb[j];
  const R a1 = T.ua[i], a2 = T.da[i], b1 = Rr * T.ub[j], b2 = Rr * T.db[j];
  const auto un = u[q + nc], us = u[q - nc], ue = u[q + 1], uw = u[q - 1], uc = u[q];
  const auto fv = f[i * nb + j];
  return mkv<R>(fv.x - (c * uc.x + a1 * un.x + a2 * us.x + b1 * ue.x + b2 * uw.x),
                fv.y - (c * uc.y + a1 * un.y + a2 * us.y + b1 * ue.y + b2 * uw.y));
}

template <typename R>
__global__ void __launch_bounds__(kThreads) k_lds_cycle(const LdsJob* __restrict__ jobs, BatchRef bt, int nu_pre,
                                                       int nu_post, int n_sor, int exact, double rtol, int max_sweeps) {
  using V = typename Vec<R>::T;
  extern __shared__ char smem[];
  __shared__ double redbuf[kThreads / 64];
  Red red{redbuf};
  const int p = blockIdx.x;
  if (bt.count && p >= *bt.count) return;
  const int e = bt.ent[p];
  const LdsJob& J = jobs[ent_prob(e)];
  const LdsLevels& LL = J.LL;
  const int slot = ent_slot(e);
  const int m = J.mode ? J.mode[slot] : slot;
  const V* __restrict__ Fg = static_cast<const V*>(J.f);
  V* __restrict__ Ug = static_cast<V*>(J.u);
  const int load_u = J.load_u;
  const int n = LL.n;
  const int cl = n - 1;  // coarsest level (FP64 storage)
  // LDS carve-up: [coarsest u, f (double2)] [levels 0..n-2 u, f (V)] [scratch (R)] [tables]
  const LevelDev& LC = LL.L[cl];
  double2* uC = reinterpret_cast<double2*>(smem);
  double2* fC = uC + (LC.na + 2) * (LC.nb + 2);
  // per-level byte offsets into LDS of u, f and the staged tables (kept in
  // LDS and turned into pointers at each use, so that the pointers stay
  // known as LDS addresses and no per-thread array is indexed dynamically)
  __shared__ int s_off[3 * kMaxLdsLevels];
  if (threadIdx.x == 0) {
    int q = (int)(sizeof(double2) * ((LC.na + 2) * (LC.nb + 2) + LC.na * LC.nb));
    for (int l = 0; l < cl; ++l) {
      s_off[l] = q;
      q += (int)sizeof(V) * (LL.L[l].na + 2) * (LL.L[l].nb + 2);
      s_off[kMaxLdsLevels + l] = q;
      q += (int)sizeof(V) * LL.L[l].na * LL.L[l].nb;
    }
    q += (int)sizeof(R) * LL.scratch;
    s_off[2 * kMaxLdsLevels + cl] = q;  // coarsest tables (double)
    q += (int)sizeof(double) * (5 * LC.na + 4 * LC.nb);
    for (int l = 0; l < cl; ++l) {
      s_off[2 * kMaxLdsLevels + l] = q;
      q += (int)sizeof(R) * (5 * LL.L[l].na + 4 * LL.L[l].nb);
    }
  }
  __syncthreads();
  auto Ul = [&](int l) { return reinterpret_cast<V*>(smem + s_off[l]); };
  auto Fl = [&](int l) { return reinterpret_cast<V*>(smem + s_off[kMaxLdsLevels + l]); };
  auto Tl = [&](int l) {
    return tab_at<R>(reinterpret_cast<R*>(smem + s_off[2 * kMaxLdsLevels + l]), LL.L[l].na, LL.L[l].nb);
  };
  R* cp = reinterpret_cast<R*>(smem + (cl > 0 ? s_off[kMaxLdsLevels + cl - 1] + (int)sizeof(V) * LL.L[cl - 1].na * LL.L[cl - 1].nb
                                               : (int)(sizeof(double2) * ((LC.na + 2) * (LC.nb + 2) + LC.na * LC.nb))));
  Tab<double> tabC = stage_tab<double>(LC, m, reinterpret_cast<double*>(smem + s_off[2 * kMaxLdsLevels + cl]));
  for (int l = 0; l < cl; ++l) (void)stage_tab<R>(LL.L[l], m, reinterpret_cast<R*>(smem + s_off[2 * kMaxLdsLevels + l]));
  // level 0 of the fused range: load f (and u for a full in-LDS cycle)
  {
    const LevelDev& L0 = LL.L[0];
    const int na = L0.na, nb = L0.nb, nc = nb + 2;
    const size_t off = (size_t)slot * na * nb;
    if (n > 1) {
      for (int t = threadIdx.x; t < (na + 2) * nc; t += blockDim.x) {
        const int i = t / nc - 1, j = t % nc - 1;
        V v = mkv<R>(0, 0);
        if (load_u && i >= 0 && i < na && j >= 0 && j < nb) v = Ug[off + (size_t)i * nb + j];
        Ul(0)[t] = v;
      }
      for (int t = threadIdx.x; t < na * nb; t += blockDim.x) Fl(0)[t] = Fg[off + t];
    } else {
      for (int t = threadIdx.x; t < na * nb; t += blockDim.x) fC[t] = make_double2(Fg[off + t].x, Fg[off + t].y);
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
    for (int k = 0; k < nu_pre; ++k) smooth_step<R>(L, T, ul, fl, n_sor, exact, cp);
    const int ncc = C.nb + 2;
    for (int t = threadIdx.x; t < (C.na + 2) * ncc; t += blockDim.x) {
      if (l + 1 == cl) uC[t] = make_double2(0.0, 0.0);
      else Ul(l + 1)[t] = mkv<R>(0, 0);
    }
    for (int t = threadIdx.x; t < C.na * C.nb; t += blockDim.x) {
      const int I = t / C.nb, J = t - I * C.nb;
      R ax = 0, ay = 0;
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
          const R w = (R)L.rwa[2 * I + a] * (R)L.rwb[2 * J + b];
          const V r = resid_lds<R>(L, T, ul, fl, 2 * I + a, 2 * J + b);
          ax = fma(w, r.x, ax);
          ay = fma(w, r.y, ay);
        }
      if (l + 1 == cl) fC[t] = make_double2(ax, ay);
      else Fl(l + 1)[t] = mkv<R>(ax, ay);
    }
    __syncthreads();
  }
  // coarsest level in FP64: the precomputed inverse when the level is small
  // (an exact solve), otherwise red-black SOR from zero until the residual
  // 2-norm dropped by rtol (Sec. 3.3)
  {
    const LevelDev& L = LC;
    const Tab<double>& T = tabC;
    const int na = L.na, nb = L.nb, nc = nb + 2;
    for (int t = threadIdx.x; t < (na + 2) * nc; t += blockDim.x) uC[t] = make_double2(0.0, 0.0);
    __syncthreads();
    if (L.cinv) {
      const int nn = na * nb;
      const double* A = L.cinv + (size_t)m * nn * nn;
      for (int k = threadIdx.x; k < nn; k += blockDim.x) {
        double sx = 0.0, sy = 0.0;
        for (int l = 0; l < nn; ++l) {
          const double a = A[(size_t)k * nn + l];
          sx = fma(a, fC[l].x, sx);
          sy = fma(a, fC[l].y, sy);
        }
        const int i = k / nb, j = k - i * nb;
        uC[(i + 1) * nc + (j + 1)] = make_double2(sx, sy);
      }
    } else {
      double f2 = 0.0;
      for (int t = threadIdx.x; t < na * nb; t += blockDim.x) f2 += fC[t].x * fC[t].x + fC[t].y * fC[t].y;
      f2 = red.sum(f2);
      const double w = L.wc[m];
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
            const double2 r = resid_lds<double>(L, T, uC, fC, i, j);
            r2 += r.x * r.x + r.y * r.y;
          }
          r2 = red.sum(r2);
          if (r2 <= rtol * rtol * f2) break;
        }
      }
    }
    __syncthreads();
  }
  // ascend
  for (int l = cl - 1; l >= 0; --l) {
    const LevelDev& L = LL.L[l];
    const LevelDev& C = LL.L[l + 1];
    const int nb = L.nb, nc = nb + 2, ncc = C.nb + 2;
    const int par = m & 1;
    const Tab<R> T = Tl(l);
    V* ul = Ul(l);
    const V* fl = Fl(l);
    for (int t = threadIdx.x; t < L.na * nb; t += blockDim.x) {
      const int i = t / nb, j = t - i * nb;
      const int a0 = L.pa_i0[i], a1 = L.pa_i1[i];
      const int b0 = L.pb_i0[par * nb + j], b1 = L.pb_i1[par * nb + j];
      const R wa0 = (R)L.pa_w0[i], wa1 = (R)L.pa_w1[i];
      const R wb0 = (R)L.pb_w0[par * nb + j], wb1 = (R)L.pb_w1[par * nb + j];
      R e00x, e00y, e01x, e01y, e10x, e10y, e11x, e11y;
      if (l + 1 == cl) {
        const double2 a = uC[(a0 + 1) * ncc + b0 + 1], b = uC[(a0 + 1) * ncc + b1 + 1];
        const double2 c = uC[(a1 + 1) * ncc + b0 + 1], d = uC[(a1 + 1) * ncc + b1 + 1];
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
    for (int k = 0; k < nu_post; ++k) smooth_step<R>(L, T, ul, fl, n_sor, exact, cp);
  }
  {
    const LevelDev& L0 = LL.L[0];
    const int na = L0.na, nb = L0.nb, nc = nb + 2;
    const size_t off = (size_t)slot * na * nb;
    for (int t = threadIdx.x; t < na * nb; t += blockDim.x) {
      const int i = t / nb, j = t - i * nb;
      if (n > 1) {
        Ug[off + t] = Ul(0)[(i + 1) * nc + (j + 1)];
      } else {
        const double2 v = uC[(i + 1) * nc + (j + 1)];
        Ug[off + t] = mkv<R>((R)v.x, (R)v.y);
      }
    }
  }
}

template <typename R>
size_t cycle_bytes(const LdsLevels& LL) {
  using V = typename Vec<R>::T;
  const int cl = LL.n - 1;
  size_t b = sizeof(double2) * ((size_t)(LL.L[cl].na + 2) * (LL.L[cl].nb + 2) + (size_t)LL.L[cl].na * LL.L[cl].nb);
  b += sizeof(double) * (5 * (size_t)LL.L[cl].na + 4 * (size_t)LL.L[cl].nb);
  for (int l = 0; l < cl; ++l) {
    b += sizeof(V) * ((size_t)(LL.L[l].na + 2) * (LL.L[l].nb + 2) + (size_t)LL.L[l].na * LL.L[l].nb);
    b += sizeof(R) * (5 * (size_t)LL.L[l].na + 4 * (size_t)LL.L[l].nb);
  }
  b += sizeof(R) * (size_t)LL.scratch;
  return b;
}

int cycle_threads(const LdsLevels& LL) {
  // enough waves that each takes about one line group per colour on the
  // first fused level; few threads keep the barriers of small levels cheap
  const int cells = LL.L[0].na * LL.L[0].nb;
  return cells >= 2048 ? 512 : (cells >= 512 ? 256 : 64);
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

size_t lds_cycle_bytes(const LdsLevels& LL, bool fp32) {
  return fp32 ? cycle_bytes<float>(LL) : cycle_bytes<double>(LL);
}

int lds_cycle_threads(const LdsLevels& LL) { return cycle_threads(LL); }

hipError_t mg_lds_cycle(const LdsJob* jobs, const LdsJob* hj, int n_prob, const BatchRef& b, int nu_pre, int nu_post,
                        int n_sor, bool exact, bool fp32, double rtol, int max_sweeps, hipStream_t st) {
  if (!b.cap) return hipSuccess;
  size_t lds = 0;
  int threads = 64;
  for (int q = 0; q < n_prob; ++q) {
    lds = std::max(lds, lds_cycle_bytes(hj[q].LL, fp32));
    threads = std::max(threads, cycle_threads(hj[q].LL));
  }
  if (lds > 64 * 1024) return hipErrorInvalidConfiguration;
  if (fp32)
    hipLaunchKernelGGL(k_lds_cycle<float>, dim3(b.cap), dim3(threads), lds, st, jobs, b, nu_pre, nu_post, n_sor,
                       exact ? 1 : 0, rtol, max_sweeps);
  else
    hipLaunchKernelGGL(k_lds_cycle<double>, dim3(b.cap), dim3(threads), lds, st, jobs, b, nu_pre, nu_post, n_sor,
                       exact ? 1 : 0, rtol, max_sweeps);
  return hipGetLastError();
}

}  // namespace smgk
