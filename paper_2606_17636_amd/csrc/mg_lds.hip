// The coarse end of the V-cycle in one launch: every level whose plane fits
// in LDS (from level `first` down to the coarsest) is processed by one block
// per plane -- pre-smoothing, residual restriction, the coarsest red-black
// SOR (Sec. 3.3), prolongation and post-smoothing -- without touching global
// memory between levels.  The arithmetic is that of the per-level kernels in
// mg.hip (same colour order, same transfer weights, same stopping rule of
// the coarsest solve); only the memory traffic and the launch count differ.
#include "smg_internal.h"

namespace {

constexpr int kThreads = 256;

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

// 1D stencil tables of one level and mode, staged in LDS.
struct Tab {
  const double *ua, *da, *R, *Ca, *wb;  // per row i
  const double *ub, *db, *Cb, *wr;      // per column j
};

__device__ Tab stage_tab(const LevelDev& L, int m, double* buf) {
  const int na = L.na, nb = L.nb;
  double* t = buf;
  for (int i = threadIdx.x; i < na; i += blockDim.x) {
    t[i] = L.ua[i];
    t[na + i] = L.da[i];
    t[2 * na + i] = L.Rr[i];
    t[3 * na + i] = L.Ca[(size_t)m * na + i];
    t[4 * na + i] = L.wb[(size_t)m * na + i];
  }
  double* c = buf + 5 * na;
  for (int j = threadIdx.x; j < nb; j += blockDim.x) {
    c[j] = L.ub[j];
    c[nb + j] = L.db[j];
    c[2 * nb + j] = L.Cb[(size_t)m * nb + j];
    c[3 * nb + j] = L.wr[(size_t)m * nb + j];
  }
  return Tab{t, t + na, t + 2 * na, t + 3 * na, t + 4 * na, c, c + nb, c + 2 * nb, c + 3 * nb};
}

// u: padded (na+2) x (nb+2) plane, f: na x nb.
template <int DIR>
__device__ void sor_phase(const LevelDev& L, const Tab& T, double2* u, const double2* f, int n_sor) {
  const int na = L.na, nb = L.nb, nc = nb + 2;
  for (int lc = 0; lc < 2; ++lc) {
    const int nl = DIR == 0 ? (nb - lc + 1) / 2 : (na - lc + 1) / 2;
    for (int it = 0; it < n_sor; ++it) {
      for (int pc = 0; pc < 2; ++pc) {
        const int np = DIR == 0 ? (na - pc + 1) / 2 : (nb - pc + 1) / 2;
        const int total = nl * np;
        for (int t = threadIdx.x; t < total; t += blockDim.x) {
          int i, j;
          if (DIR == 0) {
            i = pc + 2 * (t / nl);
            j = lc + 2 * (t % nl);
          } else {
            i = lc + 2 * (t / np);
            j = pc + 2 * (t % np);
          }
          const int q = (i + 1) * nc + (j + 1);
          const double R = T.R[i];
          const double c = T.Ca[i] + R * T.Cb[j];
          const double w = DIR == 1 ? T.wb[i] : T.wr[j];
          const double ua = T.ua[i], da = T.da[i], ub = R * T.ub[j], db = R * T.db[j];
          const double2 un = u[q + nc], us = u[q - nc], ue = u[q + 1], uw = u[q - 1];
          const double2 fv = f[i * nb + j];
          const double sx = ua * un.x + da * us.x + ub * ue.x + db * uw.x;
          const double sy = ua * un.y + da * us.y + ub * ue.y + db * uw.y;
          const double2 old = u[q];
          const double tx = (fv.x - sx) / c, ty = (fv.y - sy) / c;
          u[q] = make_double2(old.x + w * (tx - old.x), old.y + w * (ty - old.y));
        }
        __syncthreads();
      }
    }
  }
}

template <int DIR>
__device__ void exact_phase(const LevelDev& L, const Tab& T, double2* u, const double2* f, double* cp) {
  const int na = L.na, nb = L.nb, nc = nb + 2;
  const int npts = DIR == 0 ? na : nb;
  for (int lc = 0; lc < 2; ++lc) {
    const int nl = DIR == 0 ? (nb - lc + 1) / 2 : (na - lc + 1) / 2;
    for (int t = threadIdx.x; t < nl; t += blockDim.x) {
      const int line = lc + 2 * t;
      double* c1 = cp + t * npts;
      double2 prev = make_double2(0.0, 0.0);
      double cprev = 0.0;
      for (int k = 0; k < npts; ++k) {
        const int i = DIR == 1 ? line : k, j = DIR == 1 ? k : line;
        const int q = (i + 1) * nc + (j + 1);
        const double R = T.R[i];
        const double c = T.Ca[i] + R * T.Cb[j];
        double lo, up, w1, w2;
        double2 o1, o2;
        if (DIR == 1) {
          lo = R * T.db[j]; up = R * T.ub[j];
          o1 = u[q + nc]; o2 = u[q - nc]; w1 = T.ua[i]; w2 = T.da[i];
        } else {
          lo = T.da[i]; up = T.ua[i];
          o1 = u[q + 1]; o2 = u[q - 1]; w1 = R * T.ub[j]; w2 = R * T.db[j];
        }
        const double2 fv = f[i * nb + j];
        const double rx = fv.x - (w1 * o1.x + w2 * o2.x), ry = fv.y - (w1 * o1.y + w2 * o2.y);
        const double den = c - lo * cprev;
        cprev = up / den;
        c1[k] = cprev;
        prev = make_double2((rx - lo * prev.x) / den, (ry - lo * prev.y) / den);
        u[q] = prev;
      }
      for (int k = npts - 2; k >= 0; --k) {
        const int i = DIR == 1 ? line : k, j = DIR == 1 ? k : line;
        const int q = (i + 1) * nc + (j + 1);
        const double2 nx = DIR == 1 ? u[q + 1] : u[q + nc];
        const double2 d = u[q];
        u[q] = make_double2(d.x - c1[k] * nx.x, d.y - c1[k] * nx.y);
      }
    }
    __syncthreads();
  }
}

__device__ void smooth_step(const LevelDev& L, const Tab& T, double2* u, const double2* f, int n_sor, bool exact,
                            double* cp) {
  if (exact) {
    exact_phase<0>(L, T, u, f, cp);
    exact_phase<1>(L, T, u, f, cp);
  } else {
    sor_phase<0>(L, T, u, f, n_sor);
    sor_phase<1>(L, T, u, f, n_sor);
  }
}

__device__ __forceinline__ double2 resid_lds(const LevelDev& L, const Tab& T, const double2* u, const double2* f,
                                             int i, int j) {
  const int nb = L.nb, nc = nb + 2;
  const int q = (i + 1) * nc + (j + 1);
  const double R = T.R[i];
  const double c = T.Ca[i] + R * T.Cb[j];
  const double a1 = T.ua[i], a2 = T.da[i], b1 = R * T.ub[j], b2 = R * T.db[j];
  const double2 un = u[q + nc], us = u[q - nc], ue = u[q + 1], uw = u[q - 1], uc = u[q];
  const double2 fv = f[i * nb + j];
  return make_double2(fv.x - (c * uc.x + a1 * un.x + a2 * us.x + b1 * ue.x + b2 * uw.x),
                      fv.y - (c * uc.y + a1 * un.y + a2 * us.y + b1 * ue.y + b2 * uw.y));
}

__global__ void __launch_bounds__(kThreads) k_lds_cycle(LdsLevels LL, Batch bt, const double2* __restrict__ Fg,
                                                       double2* __restrict__ Ug, int load_u, int nu_pre, int nu_post,
                                                       int n_sor, int exact, double rtol, int max_sweeps) {
  extern __shared__ double2 sh[];
  __shared__ double redbuf[kThreads / 64];
  Red red{redbuf};
  const int p = blockIdx.x;
  const int slot = bt.slot[p], m = bt.mode[p];
  const int n = LL.n;
  double2* u[kMaxLdsLevels];
  double2* f[kMaxLdsLevels];
  {
    double2* q = sh;
    for (int l = 0; l < n; ++l) {
      u[l] = q; q += (LL.L[l].na + 2) * (LL.L[l].nb + 2);
      f[l] = q; q += LL.L[l].na * LL.L[l].nb;
    }
  }
  double* cp = reinterpret_cast<double*>(sh + LL.words);  // exact-line scratch
  Tab tab[kMaxLdsLevels];
  {
    double* q = cp + LL.scratch;
    for (int l = 0; l < n; ++l) {
      tab[l] = stage_tab(LL.L[l], m, q);
      q += 5 * LL.L[l].na + 4 * LL.L[l].nb;
    }
  }
  // level 0 of the fused range: load f (and u for a full in-LDS cycle)
  {
    const LevelDev& L0 = LL.L[0];
    const int na = L0.na, nb = L0.nb, nc = nb + 2;
    const size_t off = (size_t)slot * na * nb;
    for (int t = threadIdx.x; t < (na + 2) * nc; t += blockDim.x) {
      const int i = t / nc - 1, j = t % nc - 1;
      double2 v = make_double2(0.0, 0.0);
      if (load_u && i >= 0 && i < na && j >= 0 && j < nb) v = Ug[off + (size_t)i * nb + j];
      u[0][t] = v;
    }
    for (int t = threadIdx.x; t < na * nb; t += blockDim.x) f[0][t] = Fg[off + t];
  }
  __syncthreads();
  // descend
  for (int l = 0; l + 1 < n; ++l) {
    const LevelDev& L = LL.L[l];
    const LevelDev& C = LL.L[l + 1];
    for (int k = 0; k < nu_pre; ++k) smooth_step(L, tab[l], u[l], f[l], n_sor, exact, cp);
    const int ncc = C.nb + 2;
    for (int t = threadIdx.x; t < (C.na + 2) * ncc; t += blockDim.x) u[l + 1][t] = make_double2(0.0, 0.0);
    for (int t = threadIdx.x; t < C.na * C.nb; t += blockDim.x) {
      const int I = t / C.nb, J = t - I * C.nb;
      double ax = 0.0, ay = 0.0;
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
          const double w = L.rwa[2 * I + a] * L.rwb[2 * J + b];
          const double2 r = resid_lds(L, tab[l], u[l], f[l], 2 * I + a, 2 * J + b);
          ax = fma(w, r.x, ax);
          ay = fma(w, r.y, ay);
        }
      f[l + 1][t] = make_double2(ax, ay);
    }
    __syncthreads();
  }
  // coarsest: red-black SOR from zero (the same rule as k_coarse)
  {
    const LevelDev& L = LL.L[n - 1];
    const int na = L.na, nb = L.nb, nc = nb + 2;
    double2* uu = u[n - 1];
    const double2* ff = f[n - 1];
    double f2 = 0.0;
    for (int t = threadIdx.x; t < na * nb; t += blockDim.x) f2 += ff[t].x * ff[t].x + ff[t].y * ff[t].y;
    f2 = red.sum(f2);
    const double w = L.wc[m];
    if (f2 > 0.0) {
      for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        for (int colour = 0; colour < 2; ++colour) {
          for (int t = threadIdx.x; t < na * nb; t += blockDim.x) {
            const int i = t / nb, j = t - i * nb;
            if (((i + j) & 1) != colour) continue;
            const int q = (i + 1) * nc + (j + 1);
            const Tab& T = tab[n - 1];
            const double R = T.R[i];
            const double c = T.Ca[i] + R * T.Cb[j];
            const double a1 = T.ua[i], a2 = T.da[i], b1 = R * T.ub[j], b2 = R * T.db[j];
            const double2 un = uu[q + nc], us = uu[q - nc], ue = uu[q + 1], uw = uu[q - 1];
            const double2 fv = ff[t];
            const double tx = (fv.x - (a1 * un.x + a2 * us.x + b1 * ue.x + b2 * uw.x)) / c;
            const double ty = (fv.y - (a1 * un.y + a2 * us.y + b1 * ue.y + b2 * uw.y)) / c;
            const double2 old = uu[q];
            uu[q] = make_double2(old.x + w * (tx - old.x), old.y + w * (ty - old.y));
          }
          __syncthreads();
        }
        double r2 = 0.0;
        for (int t = threadIdx.x; t < na * nb; t += blockDim.x) {
          const int i = t / nb, j = t - i * nb;
          const double2 r = resid_lds(L, tab[n - 1], uu, ff, i, j);
          r2 += r.x * r.x + r.y * r.y;
        }
        r2 = red.sum(r2);
        if (r2 <= rtol * rtol * f2) break;
      }
    }
    __syncthreads();
  }
  // ascend
  for (int l = n - 2; l >= 0; --l) {
    const LevelDev& L = LL.L[l];
    const LevelDev& C = LL.L[l + 1];
    const int nb = L.nb, nc = nb + 2, ncc = C.nb + 2;
    const int par = m & 1;
    for (int t = threadIdx.x; t < L.na * nb; t += blockDim.x) {
      const int i = t / nb, j = t - i * nb;
      const int a0 = L.pa_i0[i], a1 = L.pa_i1[i];
      const int b0 = L.pb_i0[par * nb + j], b1 = L.pb_i1[par * nb + j];
      const double wa0 = L.pa_w0[i], wa1 = L.pa_w1[i];
      const double wb0 = L.pb_w0[par * nb + j], wb1 = L.pb_w1[par * nb + j];
      const double2* uc = u[l + 1];
      const double2 e00 = uc[(a0 + 1) * ncc + b0 + 1], e01 = uc[(a0 + 1) * ncc + b1 + 1];
      const double2 e10 = uc[(a1 + 1) * ncc + b0 + 1], e11 = uc[(a1 + 1) * ncc + b1 + 1];
      double ex = 0.0, ey = 0.0;
      ex = fma(wa0 * wb0, e00.x, ex); ey = fma(wa0 * wb0, e00.y, ey);
      ex = fma(wa0 * wb1, e01.x, ex); ey = fma(wa0 * wb1, e01.y, ey);
      ex = fma(wa1 * wb0, e10.x, ex); ey = fma(wa1 * wb0, e10.y, ey);
      ex = fma(wa1 * wb1, e11.x, ex); ey = fma(wa1 * wb1, e11.y, ey);
      const int q = (i + 1) * nc + (j + 1);
      u[l][q] = make_double2(u[l][q].x + ex, u[l][q].y + ey);
    }
    __syncthreads();
    for (int k = 0; k < nu_post; ++k) smooth_step(L, tab[l], u[l], f[l], n_sor, exact, cp);
  }
  {
    const LevelDev& L0 = LL.L[0];
    const int na = L0.na, nb = L0.nb, nc = nb + 2;
    const size_t off = (size_t)slot * na * nb;
    for (int t = threadIdx.x; t < na * nb; t += blockDim.x) {
      const int i = t / nb, j = t - i * nb;
      Ug[off + t] = u[0][(i + 1) * nc + (j + 1)];
    }
  }
}

}  // namespace

namespace smgk {

size_t lds_cycle_bytes(const LdsLevels& LL, bool exact) {
  size_t words = 0, scratch = 0, tabs = 0;
  for (int l = 0; l < LL.n; ++l) {
    words += (size_t)(LL.L[l].na + 2) * (LL.L[l].nb + 2) + (size_t)LL.L[l].na * LL.L[l].nb;
    tabs += 5 * (size_t)LL.L[l].na + 4 * (size_t)LL.L[l].nb;
    if (exact) {
      const size_t a = (size_t)((LL.L[l].nb + 1) / 2) * LL.L[l].na;
      const size_t b = (size_t)((LL.L[l].na + 1) / 2) * LL.L[l].nb;
      scratch = scratch > a ? scratch : a;
      scratch = scratch > b ? scratch : b;
    }
  }
  return words * sizeof(double2) + (scratch + tabs) * sizeof(double);
}

int lds_cycle_scratch(const LdsLevels& LL, bool exact) {
  size_t scratch = 0;
  if (exact)
    for (int l = 0; l < LL.n; ++l) {
      const size_t a = (size_t)((LL.L[l].nb + 1) / 2) * LL.L[l].na;
      const size_t b = (size_t)((LL.L[l].na + 1) / 2) * LL.L[l].nb;
      scratch = scratch > a ? scratch : a;
      scratch = scratch > b ? scratch : b;
    }
  return (int)scratch;
}

hipError_t mg_lds_cycle(const LdsLevels& LL, const Batch& b, const double2* f, double2* u, bool load_u, int nu_pre,
                        int nu_post, int n_sor, bool exact, double rtol, int max_sweeps, hipStream_t st) {
  if (b.n == 0) return hipSuccess;
  // the fused levels are small: a single wavefront per plane makes every
  // colour-step barrier nearly free
  const int threads = LL.L[0].na * LL.L[0].nb >= 2048 ? 256 : (LL.L[0].na * LL.L[0].nb >= 512 ? 128 : 64);
  hipLaunchKernelGGL(k_lds_cycle, dim3(b.n), dim3(threads), lds_cycle_bytes(LL, exact), st, LL, b, f, u,
                     load_u ? 1 : 0, nu_pre, nu_post, n_sor, exact ? 1 : 0, rtol, max_sweeps);
  return hipGetLastError();
}

}  // namespace smgk
