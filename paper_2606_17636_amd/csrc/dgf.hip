// One-time construction of the discrete Green's function tables (Sec. 4.2).
//
// Gt^m(t <- s) = G^m(t <- s) * dV_s (dV_s: full 3D volume of source ghost s)
// solves L_m Gt = 4 pi G e_s on a box of cells around the source with
//   * Dirichlet ring values dV_s * Gc^m, Gc^m(x, x') = -G sum_{k<N}
//     cos(2 pi m k / N) / |x - x'(phi_k)|   (Eqs. DGF_bc_sph / DGF_bc_cyl),
//   * on a Neumann inner radial edge the flux A dGc^m/dr (derivative formulas
//     of Sec. 4.2), evaluated on the edge face,
//   * pole parity where the box reaches a pole.
// Two boxes are used: the auxiliary grid of (2 n_pad + 1)^2 cells around
// each source (uniform radial grids; solved here by red-black SOR in LDS,
// one block per (mode, source)), and the extended domain shared by all
// sources (logarithmic radial grids; solved by the batched multigrid, two
// real sources per complex plane).  Field ghosts inside a box take the
// solved value, the others dV_s * Gc^m.
#include "dgf_dev.h"

namespace {

constexpr int kThreads = 256;
constexpr double kFourPi = 12.566370614359172953850573533118;
constexpr double kPi = 3.141592653589793238462643383279502884;

}  // namespace

// -- continuous-kernel Fourier coefficients -----------------------------------
__device__ double kernel_sum(const DgfConst& K, int m, double a, double b, double as, double bs) {
  double acc = 0.0;
  if (K.sph) {
    const double A = a * a + as * as - 2.0 * a * as * cos(b) * cos(bs);
    const double B = 2.0 * a * as * sin(b) * sin(bs);
    for (int k = 0; k < K.n_phi; ++k) {
      const double d2 = A - B * K.cosk[k];
      acc += K.cosk[(int)(((long)m * k) % K.n_phi)] / sqrt(d2);
    }
  } else {
    const double A = a * a + as * as + (b - bs) * (b - bs);
    const double B = 2.0 * a * as;
    for (int k = 0; k < K.n_phi; ++k) {
      const double d2 = A - B * K.cosk[k];
      acc += K.cosk[(int)(((long)m * k) % K.n_phi)] / sqrt(d2);
    }
  }
  return -K.G * acc;
}

__device__ double kernel_dr_sum(const DgfConst& K, int m, double a, double b, double as, double bs) {
  double acc = 0.0;
  if (K.sph) {
    const double A = a * a + as * as - 2.0 * a * as * cos(b) * cos(bs);
    const double B = 2.0 * a * as * sin(b) * sin(bs);
    const double C = a - as * cos(b) * cos(bs);
    const double D = as * sin(b) * sin(bs);
    for (int k = 0; k < K.n_phi; ++k) {
      const double ck = K.cosk[k];
      const double d2 = A - B * ck;
      acc += (C - D * ck) * K.cosk[(int)(((long)m * k) % K.n_phi)] / (d2 * sqrt(d2));
    }
  } else {
    const double A = a * a + as * as + (b - bs) * (b - bs);
    const double B = 2.0 * a * as;
    for (int k = 0; k < K.n_phi; ++k) {
      const double ck = K.cosk[k];
      const double d2 = A - B * ck;
      acc += (a - as * ck) * K.cosk[(int)(((long)m * k) % K.n_phi)] / (d2 * sqrt(d2));
    }
  }
  return K.G * acc;
}

namespace {

__device__ double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
  return s;
}

// Auxiliary-grid DGF: block (p, s) solves the box of source s for mode
// modes[p] and writes column s of table p.
__global__ void __launch_bounds__(kThreads) k_dgf_aux(DgfConst K, AuxBoxes X, const int* __restrict__ modes,
                                                     double* __restrict__ out, double tol, int max_sweeps,
                                                     double* __restrict__ resid_out) {
  extern __shared__ double lds[];
  __shared__ double red[kThreads / 64];
  const int p = blockIdx.y, s = blockIdx.x;
  const int m = modes[p];
  const int i_lo = X.i_lo[s], i_hi = X.i_hi[s], j_lo = X.j_lo[s], j_hi = X.j_hi[s];
  const int e_alo = X.e_alo[s], e_blo = X.e_blo[s], e_bhi = X.e_bhi[s];
  const int n1 = i_hi - i_lo + 1, n2 = j_hi - j_lo + 1;
  const int ld = n2 + 2;
  double* u = lds;                      // (n1+2) x (n2+2), zero border
  double* rhs = u + (n1 + 2) * ld;      // n1 x n2
  double* cu = rhs + n1 * n2;           // per-row coefficients: ua, da, R, Ca
  double* cd = cu + n1;
  double* cr = cd + n1;
  double* ca = cr + n1;
  double* bu = ca + n1;                 // per-column: ub, db, Cb
  double* bd = bu + n2;
  double* cb = bd + n2;
  const double s2 = K.s2[m];
  const double kap_lo = e_blo == 1 ? ((m & 1) ? -1.0 : 1.0) : 0.0;
  const double kap_hi = e_bhi == 1 ? ((m & 1) ? -1.0 : 1.0) : 0.0;
  for (int i = threadIdx.x; i < n1; i += blockDim.x) {
    const int k = i_lo + i - X.offA;
    const double up = X.upA[k], dn = X.dnA[k];
    cu[i] = (i == n1 - 1) ? 0.0 : up;
    cd[i] = (i == 0) ? 0.0 : dn;
    const double dneff = (i == 0 && e_alo == 2) ? 0.0 : dn;
    double c = -(up + dneff);
    if (!K.sph) c -= s2 * X.PA[k];
    ca[i] = c;
    cr[i] = K.sph ? X.RA[k] : 1.0;
  }
  for (int j = threadIdx.x; j < n2; j += blockDim.x) {
    const int k = j_lo + j - X.offB;
    const double up = X.upB[k], dn = X.dnB[k];
    bu[j] = (j == n2 - 1) ? 0.0 : up;
    bd[j] = (j == 0) ? 0.0 : dn;
    double c = -(up + dn);
    if (j == 0) c += kap_lo * dn;
    if (j == n2 - 1) c += kap_hi * up;
    if (K.sph) c -= s2 * X.PB[k];
    cb[j] = c;
  }
  for (int t = threadIdx.x; t < (n1 + 2) * ld; t += blockDim.x) u[t] = 0.0;
  __syncthreads();
  // right-hand side: unit source plus folded boundary data
  const double as = X.ga[s], bs = X.gb[s], dvs = X.gdv[s];
  for (int t = threadIdx.x; t < n1 * n2; t += blockDim.x) {
    const int i = t / n2, j = t - i * n2;
    const int ka = i_lo + i - X.offA, kb = j_lo + j - X.offB;
    double r = 0.0;
    if (i_lo + i == X.gi[s] && j_lo + j == X.gj[s]) r += kFourPi * K.G;
    if (i == 0) {
      if (e_alo == 0)
        r -= X.dnA[ka] * dvs * kernel_sum(K, m, X.centA[ka - 1], X.centB[kb], as, bs);
      else
        r += X.nfA[ka] * dvs * kernel_dr_sum(K, m, X.faceA[ka], X.centB[kb], as, bs);
    }
    if (i == n1 - 1) r -= X.upA[ka] * dvs * kernel_sum(K, m, X.centA[ka + 1], X.centB[kb], as, bs);
    const double R = K.sph ? X.RA[ka] : 1.0;
    if (j == 0 && e_blo == 0) r -= R * X.dnB[kb] * dvs * kernel_sum(K, m, X.centA[ka], X.centB[kb - 1], as, bs);
    if (j == n2 - 1 && e_bhi == 0) r -= R * X.upB[kb] * dvs * kernel_sum(K, m, X.centA[ka], X.centB[kb + 1], as, bs);
    rhs[t] = r;
  }
  __syncthreads();
  // 2D WKB omega of the box (p = q = 1 term of Appendix A)
  double num = 0.0, den = 0.0;
  {
    const int ka0 = i_lo - X.offA, kb0 = j_lo - X.offB;
    const double x0 = (e_alo == 2) ? X.faceA[ka0] : X.centA[ka0 - 1];
    const double La = X.centA[ka0 + n1] - x0;
    const double y0 = X.centB[kb0 - 1];
    const double Lb = X.centB[kb0 + n2] - y0;
    for (int t = threadIdx.x; t < n1 * n2; t += blockDim.x) {
      const int i = t / n2, j = t - i * n2;
      const double xa = X.centA[ka0 + i], xam = (i == 0) ? x0 : X.centA[ka0 + i - 1];
      const double yb = X.centB[kb0 + j], ybm = X.centB[kb0 + j - 1];
      double wa = sin(kPi * (xa - x0) / La), wb = sin(kPi * (yb - y0) / Lb);
      const double w = wa * wa * wb * wb;
      num += ((cu[i] + cd[i]) * cos(kPi * (xa - xam) / La) + cr[i] * (bu[j] + bd[j]) * cos(kPi * (yb - ybm) / Lb)) * w;
      den += (ca[i] + cr[i] * cb[j]) * w;
    }
  }
  num = block_sum(num, red);
  den = block_sum(den, red);
  double rho = fabs(num / den);
  if (rho > 1.0) rho = 1.0;
  const double omega = 2.0 / (1.0 + sqrt(fmax(0.0, 1.0 - rho * rho)));
  double f2 = 0.0;
  for (int t = threadIdx.x; t < n1 * n2; t += blockDim.x) f2 += rhs[t] * rhs[t];
  f2 = block_sum(f2, red);
  int sweep = 0;
  double rel = f2 > 0.0 ? 1.0 : 0.0;
  for (; sweep < max_sweeps && f2 > 0.0; ++sweep) {
    for (int colour = 0; colour < 2; ++colour) {
      for (int t = threadIdx.x; t < n1 * n2; t += blockDim.x) {
        const int i = t / n2, j = t - i * n2;
        if (((i + j) & 1) != colour) continue;
        const int q = (i + 1) * ld + (j + 1);
        const double R = cr[i];
        const double c = ca[i] + R * cb[j];
        const double nbs = cu[i] * u[q + ld] + cd[i] * u[q - ld] + R * (bu[j] * u[q + 1] + bd[j] * u[q - 1]);
        const double v = (rhs[t] - nbs) / c;
        u[q] += omega * (v - u[q]);
      }
      __syncthreads();
    }
    if ((sweep & 7) == 7) {
      double r2 = 0.0;
      for (int t = threadIdx.x; t < n1 * n2; t += blockDim.x) {
        const int i = t / n2, j = t - i * n2;
        const int q = (i + 1) * ld + (j + 1);
        const double R = cr[i];
        const double c = ca[i] + R * cb[j];
        const double r = rhs[t] - (c * u[q] + cu[i] * u[q + ld] + cd[i] * u[q - ld] + R * (bu[j] * u[q + 1] + bd[j] * u[q - 1]));
        r2 += r * r;
      }
      r2 = block_sum(r2, red);
      rel = sqrt(r2 / f2);
      if (rel <= tol) break;
    }
  }
  if (threadIdx.x == 0) resid_out[(size_t)p * gridDim.x + s] = rel;
  // column s: solved values inside the box, the continuous kernel elsewhere
  double* col = out + (size_t)p * K.n_g * K.n_g;
  for (int t = threadIdx.x; t < K.n_g; t += blockDim.x) {
    const int gi = X.gi[t], gj = X.gj[t];
    double v;
    if (gi >= i_lo && gi <= i_hi && gj >= j_lo && gj <= j_hi) {
      v = u[(gi - i_lo + 1) * ld + (gj - j_lo + 1)];
    } else {
      v = dvs * kernel_sum(K, m, X.ga[t], X.gb[t], as, bs);
    }
    col[(size_t)t * K.n_g + s] = v;
  }
}

// Extended domain: right-hand sides of a chunk of planes.  Plane q holds
// sources src0[q] (real part) and src1[q] (imaginary part, -1 if none).
__global__ void k_dgf_ext_boundary(DgfConst K, ExtBox E, const int* __restrict__ pmode,
                                   const int* __restrict__ src0, const int* __restrict__ src1,
                                   double2* __restrict__ f) {
  const int q = blockIdx.y;
  const int m = pmode[q];
  const int na = E.na, nb = E.nb;
  const int nper = 2 * (na + nb);
  double2* fq = f + (size_t)q * na * nb;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nper; t += gridDim.x * blockDim.x) {
    // enumerate perimeter cells without duplicates: rows 0 and na-1 fully,
    // then columns 0 and nb-1 for the rows in between
    int i, j;
    if (t < nb) { i = 0; j = t; }
    else if (t < 2 * nb) { i = na - 1; j = t - nb; }
    else if (t < 2 * nb + (na - 2)) { i = 1 + (t - 2 * nb); j = 0; }
    else if (t < 2 * nb + 2 * (na - 2)) { i = 1 + (t - 2 * nb - (na - 2)); j = nb - 1; }
    else continue;
    double2 acc = make_double2(0.0, 0.0);
    for (int h = 0; h < 2; ++h) {
      const int s = h == 0 ? src0[q] : src1[q];
      if (s < 0) continue;
      const double as = E.ga[s], bs = E.gb[s], dvs = E.gdv[s];
      double v = 0.0;
      const double R = K.sph ? E.RA[i] : 1.0;
      if (i == 0) v += E.nfA * dvs * kernel_dr_sum(K, m, E.face0, E.centB[j + 1], as, bs);  // Neumann inner edge
      if (i == na - 1) v -= E.upA_last * dvs * kernel_sum(K, m, E.centA[na + 1], E.centB[j + 1], as, bs);
      if (j == 0 && E.e_blo == 0) v -= R * E.dnB_first * dvs * kernel_sum(K, m, E.centA[i + 1], E.centB[0], as, bs);
      if (j == nb - 1 && E.e_bhi == 0) v -= R * E.upB_last * dvs * kernel_sum(K, m, E.centA[i + 1], E.centB[nb + 1], as, bs);
      if (h == 0) acc.x += v; else acc.y += v;
    }
    fq[(size_t)i * nb + j] = acc;
  }
}

__global__ void k_dgf_ext_sources(DgfConst K, ExtBox E, const int* __restrict__ src0, const int* __restrict__ src1,
                                  int nplanes, double2* __restrict__ f) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nplanes) return;
  double2* fq = f + (size_t)q * E.na * E.nb;
  const int s0 = src0[q], s1 = src1[q];
  fq[E.cell[s0]].x += kFourPi * K.G;
  if (s1 >= 0) fq[E.cell[s1]].y += kFourPi * K.G;
}

__global__ void k_dgf_ext_extract(ExtBox E, int n_g, const int* __restrict__ ptab, const int* __restrict__ src0,
                                  const int* __restrict__ src1, const double2* __restrict__ u,
                                  double* __restrict__ out) {
  const int q = blockIdx.y;
  const double2* uq = u + (size_t)q * E.na * E.nb;
  double* tab = out + (size_t)ptab[q] * n_g * n_g;
  const int s0 = src0[q], s1 = src1[q];
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n_g; t += gridDim.x * blockDim.x) {
    const double2 v = uq[E.cell[t]];
    tab[(size_t)t * n_g + s0] = v.x;
    if (s1 >= 0) tab[(size_t)t * n_g + s1] = v.y;
  }
}

}  // namespace

namespace smgk {

hipError_t dgf_aux(const DgfConst& K, const AuxBoxes& X, const int* modes, int n_modes, double* out, double tol,
                   int max_sweeps, double* resid, int max_n1, int max_n2, hipStream_t st) {
  const size_t lds = sizeof(double) * ((size_t)(max_n1 + 2) * (max_n2 + 2) + (size_t)max_n1 * max_n2 +
                                       4 * (size_t)max_n1 + 3 * (size_t)max_n2);
  hipLaunchKernelGGL(k_dgf_aux, dim3(K.n_g, n_modes), dim3(kThreads), lds, st, K, X, modes, out, tol, max_sweeps,
                     resid);
  return hipGetLastError();
}

hipError_t dgf_ext_rhs(const DgfConst& K, const ExtBox& E, const int* pmode, const int* src0, const int* src1,
                       int nplanes, double2* f, hipStream_t st) {
  hipError_t e = fill_zero(f, (size_t)nplanes * E.na * E.nb, st);
  if (e != hipSuccess) return e;
  const int nper = 2 * (E.na + E.nb);
  hipLaunchKernelGGL(k_dgf_ext_boundary, dim3((nper + 255) / 256, nplanes), dim3(256), 0, st, K, E, pmode, src0,
                     src1, f);
  hipLaunchKernelGGL(k_dgf_ext_sources, dim3((nplanes + 255) / 256), dim3(256), 0, st, K, E, src0, src1, nplanes, f);
  return hipGetLastError();
}

hipError_t dgf_ext_extract(const ExtBox& E, int n_g, const int* ptab, const int* src0, const int* src1, int nplanes,
                           const double2* u, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_dgf_ext_extract, dim3((n_g + 255) / 256, nplanes), dim3(256), 0, st, E, n_g, ptab, src0, src1,
                     u, out);
  return hipGetLastError();
}

}  // namespace smgk
