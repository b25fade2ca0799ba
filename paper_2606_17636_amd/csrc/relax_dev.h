// Zebra line relaxation with the lines held in registers (Sec. 3.2,
// Algorithm 1; even-odd ordering inside a line as in Sec. 5.2).
//
// One colour of one direction: the lines a, a+2, ... < b are relaxed by
// n_sor even-odd SOR passes each.  The neighbouring lines (the other colour)
// do not change during the colour, so their contribution is folded into the
// right-hand side once, and omega / diagonal is formed once per cell.  A
// line belongs to a contiguous run of lanes of one wave, P consecutive
// points per lane (P even, so a lane's point s has the parity of s); the
// only neighbour a pass needs from outside the lane comes from the adjacent
// lane by a DPP wave shift, so the passes of a colour touch neither LDS nor
// a barrier.  u is read from and written back to LDS once per colour.
//
// Update of point p with neighbours p-1, p+1 along the line (lo_p, up_p the
// couplings, c_p the diagonal, rhs_p = f_p minus the across-line terms):
//   u_p <- (1 - omega) u_p + (omega / c_p) (rhs_p - lo_p u_{p-1} - up_p u_{p+1})
// which is the over-relaxed Gauss-Seidel step u_p + omega (t_p - u_p) with
// t_p the point's exact solve.  Couplings that leave the plane are zero in
// the tables (boundary data live in f), and points past the end of a line
// are never stored.
#pragma once

#include "vec.h"

// Where a block finds u, f and the 1D stencil tables of one plane: u(i, j) =
// u[(i + ui) * us + j + uj], f(i, j) = f[(i + fi) * fs + j + fj], row tables
// at [i + ti], column tables at [j + tj] (all offsets make the indices of
// the cells a block touches non-negative).
template <typename R>
struct LineView {
  typename Vec<R>::T* u;
  int us, ui, uj;
  const typename Vec<R>::T* f;
  int fs, fi, fj;
  const R *ua, *da, *Rr, *Ca, *wb;  // per row i: couplings to i+1, i-1, metric factor, diagonal part, polar-line omega
  int ti;
  const R *ub, *db, *Cb, *wr;       // per column j: couplings to j+1, j-1, diagonal part, radial-line omega
  int tj;
};

// value of lane l-1 (zero in lane 0) / of lane l+1 (zero in lane 63)
__device__ __forceinline__ float lane_prev(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float lane_next(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ double lane_prev(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), 0x138, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x138, 0xf, 0xf, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double lane_next(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), 0x130, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x130, 0xf, 0xf, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Row strides of the LDS planes that the line kernels use: odd, so that the
// lanes of a wave walking down a column (radial lines) hit distinct banks.
__host__ __device__ __forceinline__ int odd_stride(int n) { return n | 1; }

// Points per lane for lines of npts points: the smallest of 2, 4, 8, 16
// with npts <= 64 P, so that a line fits in one wave (lines longer than
// kRelaxMaxPoints are rejected when a plan is made).
constexpr int kRelaxMaxPoints = 1024;
__host__ __device__ __forceinline__ int relax_points_per_lane(int npts) {
  return npts <= 128 ? 2 : (npts <= 256 ? 4 : (npts <= 512 ? 8 : 16));
}

// omega / c: exact in FP64; in the FP32 smoothing of the mixed form the
// hardware reciprocal (within 1 ulp), which changes the smoother's weights
// by about one FP32 rounding.
__device__ __forceinline__ float omega_over(float om, float c) { return om * __builtin_amdgcn_rcpf(c); }
__device__ __forceinline__ double omega_over(double om, double c) { return om / c; }

// DIR = 1: polar lines (fixed row i, points j); DIR = 0: radial lines (fixed
// column j, points i).  Every thread of the block calls this; waves take
// groups of lines in turn.  Lanes past the last line or point load a valid
// cell instead (clamped indices) and store nothing: their values never
// reach a stored point, since the couplings across a line's ends are zero
// and the segment ends are masked in the shifts.
template <int DIR, int P, typename R>
__device__ __forceinline__ void relax_colour_p(const LineView<R>& v, int a, int b, int npts, int n_sor) {
  using V = typename Vec<R>::T;
  const int lpl = (npts + P - 1) / P;  // lanes per line
  if (lpl > 64) return;                // longer than kRelaxMaxPoints: never planned
  const int G = 64 / lpl;              // lines per wave step
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
  const int g = lane / lpl, k = lane - g * lpl;
  const int nl = a < b ? (b - a + 1) / 2 : 0;
  const bool first = k == 0, last = k == lpl - 1;
  for (int base = wave * G; base < nl; base += nwave * G) {  // uniform in the wave
    const int li = base + g;
    const bool act = g < G && li < nl;
    const int line = a + 2 * (act ? li : 0);
    R ux[P], uy[P], rx[P], ry[P], wc[P], lo[P], up[P];
    R omc;
    if (DIR == 1) {
      const int ti = line + v.ti;
      const R om = v.wb[ti], a1 = v.ua[ti], a2 = v.da[ti], rr = v.Rr[ti], ca = v.Ca[ti];
      omc = (R)1 - om;
      const V* ur = v.u + (line + v.ui) * v.us + v.uj;
      const V* fr = v.f + (line + v.fi) * v.fs + v.fj;
#pragma unroll
      for (int s = 0; s < P; ++s) {
        const int j = min(P * k + s, npts - 1);
        const int tj = j + v.tj;
        lo[s] = rr * v.db[tj];
        up[s] = rr * v.ub[tj];
        wc[s] = omega_over(om, ca + rr * v.Cb[tj]);
        const V uc = ur[j], un = ur[j + v.us], us = ur[j - v.us], fv = fr[j];
        ux[s] = uc.x; uy[s] = uc.y;
        rx[s] = fv.x - (a1 * un.x + a2 * us.x);
        ry[s] = fv.y - (a1 * un.y + a2 * us.y);
      }
    } else {
      const int j = line, tj = j + v.tj;
      const R om = v.wr[tj], b1 = v.ub[tj], b2 = v.db[tj], cb = v.Cb[tj];
      omc = (R)1 - om;
#pragma unroll
      for (int s = 0; s < P; ++s) {
        const int i = min(P * k + s, npts - 1);
        const int ti = i + v.ti;
        const R rr = v.Rr[ti];
        lo[s] = v.da[ti];
        up[s] = v.ua[ti];
        wc[s] = omega_over(om, v.Ca[ti] + rr * cb);
        const V* uq = v.u + (i + v.ui) * v.us + j + v.uj;
        const V uc = uq[0], ue = uq[1], uw = uq[-1];
        const V fv = v.f[(i + v.fi) * v.fs + j + v.fj];
        ux[s] = uc.x; uy[s] = uc.y;
        rx[s] = fv.x - rr * (b1 * ue.x + b2 * uw.x);
        ry[s] = fv.y - rr * (b1 * ue.y + b2 * uw.y);
      }
    }
    for (int it = 0; it < n_sor; ++it) {
      // even points: the left neighbour of point 0 is the last point of lane k-1
      {
        R lx = lane_prev(ux[P - 1]), ly = lane_prev(uy[P - 1]);
        if (first) lx = ly = 0;
#pragma unroll
        for (int s = 0; s < P; s += 2) {
          const R px = s > 0 ? ux[s - 1] : lx, py = s > 0 ? uy[s - 1] : ly;
          const R nx = ux[s + 1], ny = uy[s + 1];
          ux[s] = omc * ux[s] + wc[s] * (rx[s] - lo[s] * px - up[s] * nx);
          uy[s] = omc * uy[s] + wc[s] * (ry[s] - lo[s] * py - up[s] * ny);
        }
      }
      // odd points: the right neighbour of point P-1 is the first point of lane k+1
      {
        R qx = lane_next(ux[0]), qy = lane_next(uy[0]);
        if (last) qx = qy = 0;
#pragma unroll
        for (int s = 1; s < P; s += 2) {
          const R px = ux[s - 1], py = uy[s - 1];
          const R nx = s < P - 1 ? ux[s + 1] : qx, ny = s < P - 1 ? uy[s + 1] : qy;
          ux[s] = omc * ux[s] + wc[s] * (rx[s] - lo[s] * px - up[s] * nx);
          uy[s] = omc * uy[s] + wc[s] * (ry[s] - lo[s] * py - up[s] * ny);
        }
      }
    }
    if (act) {
#pragma unroll
      for (int s = 0; s < P; ++s) {
        const int pt = P * k + s;
        if (pt < npts) {
          const int i = DIR == 1 ? line : pt, j = DIR == 1 ? pt : line;
          v.u[(i + v.ui) * v.us + j + v.uj] = mkv<R>(ux[s], uy[s]);
        }
      }
    }
  }
}

// Dispatch on the points per lane of this line length, for kernels built
// for lines of up to 64 PMAX points (the launcher picks PMAX from the longest
// line it relaxes, so the register footprint is that of PMAX).
template <int DIR, int PMAX, typename R>
__device__ __forceinline__ void relax_colour(const LineView<R>& v, int a, int b, int npts, int n_sor) {
  const int P = relax_points_per_lane(npts);
  if constexpr (PMAX >= 16) {
    if (P == 16) { relax_colour_p<DIR, 16, R>(v, a, b, npts, n_sor); return; }
  }
  if constexpr (PMAX >= 8) {
    if (P == 8) { relax_colour_p<DIR, 8, R>(v, a, b, npts, n_sor); return; }
  }
  if constexpr (PMAX >= 4) {
    if (P == 4) { relax_colour_p<DIR, 4, R>(v, a, b, npts, n_sor); return; }
  }
  relax_colour_p<DIR, 2, R>(v, a, b, npts, n_sor);
}
