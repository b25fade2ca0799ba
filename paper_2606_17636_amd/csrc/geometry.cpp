// Host-side plan tables: finite-volume geometry (Sec. 2.1.1, Sec. 2.1.2),
// per-mode Helmholtz stencil factors (Sec. 2.2), WKB over-relaxation
// parameters (Appendix A), grid-transfer weights (Sec. 3.1) and the James
// ghost-cell set (Sec. 4.1).  Everything here is one-time FP64 setup.
//
// Conventions (see smg_internal.h): an axis has interior cells 1..n and one
// ghost cell each side; ghosts continue the face law of their level, a ghost
// across a pole is the mirror cell, faces on a pole have zero sine.  The
// operator diagonal is split as c_ij = Ca[m][i] + Rr[i] * Cb[m][j]; ghost
// couplings are removed from the off-diagonals and ghosts that are a fixed
// multiple kappa of the adjacent cell (pole parity (-1)^m, Neumann +1) are
// folded into the diagonal.  On coarse multigrid levels a Dirichlet ghost is
// such a multiple too: the homogeneous error condition stays at the finest
// level's ghost centre, so the coarse ghost is the value that the straight
// line through it and the first coarse centre takes there.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>

#include "smg_internal.h"

namespace smg {

static const double kPi = 3.141592653589793238462643383279502884;

std::string strprintf(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  return std::string(buf);
}

bool Spec::pole_lo() const { return sph() && b_min == 0.0; }
bool Spec::pole_hi() const { return sph() && std::fabs(b_max - kPi) < 1e-12; }
double Spec::dphi() const { return 2.0 * kPi / n_phi; }

double Spec::radial_face(double f) const {
  if (radial == SMG_RADIAL_UNIFORM) return a_min + f * ((a_max - a_min) / n_a);
  return a_min * std::pow(a_max / a_min, f / n_a);
}

bool Spec::b_face_is_pole(long f) const {
  return (pole_lo() && f == 0) || (pole_hi() && f == n_b);
}

double Spec::b_face(long f) const {
  if (pole_lo() && f == 0) return 0.0;
  if (pole_hi() && f == n_b) return kPi;
  return b_min + (double)f * ((b_max - b_min) / n_b);
}

double mode_s2(int n_phi, int m) {
  double s = std::sin(m * kPi / n_phi) / (kPi / n_phi);
  return s * s;
}

double kappa(int kind, int m) {
  if (kind == EDGE_DIRICHLET) return 0.0;
  if (kind == EDGE_POLE) return (m % 2) ? -1.0 : 1.0;
  return 1.0;  // Neumann
}

Axis make_axis(const Spec& s, char which, long off, long stride, int n) {
  Axis ax;
  ax.which = which;
  ax.n = n;
  ax.off = off;
  ax.stride = stride;
  ax.face.resize(n + 3);
  ax.sinf.assign(n + 3, 0.0);
  std::vector<bool> pole(n + 3, false);
  for (int q = 0; q < n + 3; ++q) {
    long f = off + (long)(q - 1) * stride;
    if (which == 'a') {
      ax.face[q] = s.radial_face((double)f);
    } else {
      ax.face[q] = s.b_face(f);
      pole[q] = s.b_face_is_pole(f);
      if (s.sph()) ax.sinf[q] = pole[q] ? 0.0 : std::sin(ax.face[q]);
    }
  }
  ax.pole_lo = which == 'b' && pole[1];
  ax.pole_hi = which == 'b' && pole[n + 1];
  ax.cent.resize(n + 2);
  ax.vol.resize(n + 2);
  for (int k = 0; k < n + 2; ++k) {
    double lo = ax.face[k], hi = ax.face[k + 1];
    if (which == 'a') {
      if (s.sph()) {
        ax.cent[k] = 0.75 * (hi * hi * hi * hi - lo * lo * lo * lo) / (hi * hi * hi - lo * lo * lo);
        ax.vol[k] = (hi * hi * hi - lo * lo * lo) / 3.0;
      } else {
        ax.cent[k] = (2.0 / 3.0) * (hi * hi * hi - lo * lo * lo) / (hi * hi - lo * lo);
        ax.vol[k] = 0.5 * (hi * hi - lo * lo);
      }
    } else {
      if (s.sph()) {
        ax.cent[k] = (std::sin(hi) - std::sin(lo) + lo * std::cos(lo) - hi * std::cos(hi)) /
                     (std::cos(lo) - std::cos(hi));
        ax.vol[k] = std::cos(lo) - std::cos(hi);
      } else {
        ax.cent[k] = 0.5 * (lo + hi);
        ax.vol[k] = hi - lo;
      }
    }
  }
  if (ax.pole_lo) ax.cent[0] = -ax.cent[1];
  if (ax.pole_hi) ax.cent[n + 1] = 2.0 * kPi - ax.cent[n];
  ax.up.assign(n + 2, 0.0);
  ax.dn.assign(n + 2, 0.0);
  ax.R.assign(n + 2, 1.0);
  ax.P.assign(n + 2, 1.0);
  for (int k = 0; k < n + 2; ++k) {
    double lo = ax.face[k], hi = ax.face[k + 1], x = ax.cent[k];
    double xp = ax.cent[k + 1 < n + 2 ? k + 1 : k], xm = ax.cent[k > 0 ? k - 1 : k];
    if (which == 'a') {
      if (s.sph()) {
        double den = hi * hi * hi - lo * lo * lo;
        if (k < n + 1) ax.up[k] = 3.0 * hi * hi / (den * (xp - x));
        if (k > 0) ax.dn[k] = 3.0 * lo * lo / (den * (x - xm));
        ax.R[k] = 1.5 / x * (hi * hi - lo * lo) / den;
        ax.P[k] = ax.R[k];
      } else {
        double den = hi * hi - lo * lo;
        if (k < n + 1) ax.up[k] = 2.0 * hi / (den * (xp - x));
        if (k > 0) ax.dn[k] = 2.0 * lo / (den * (x - xm));
        ax.P[k] = 2.0 / (x * (hi + lo));
      }
    } else {
      if (s.sph()) {
        double den = std::cos(lo) - std::cos(hi);
        if (k < n + 1) ax.up[k] = ax.sinf[k + 1] / (den * (xp - x));
        if (k > 0) ax.dn[k] = ax.sinf[k] / (den * (x - xm));
        ax.P[k] = (hi - lo) / (std::sin(x) * den);
      } else {
        double den = hi - lo;
        if (k < n + 1) ax.up[k] = 1.0 / (den * (xp - x));
        if (k > 0) ax.dn[k] = 1.0 / (den * (x - xm));
      }
    }
  }
  return ax;
}

// WKB Jacobi radius of a tridiagonal line (Appendix A): positions x[0..n+1]
// (including the two end positions), couplings and diagonal of points 1..n.
static double wkb_radius(const double* x, int n, const double* lower, const double* upper,
                         const double* diag, int dstride) {
  double L = x[n + 1] - x[0];
  double num = 0.0, den = 0.0;
  for (int k = 1; k <= n; ++k) {
    double w = std::sin(kPi * (x[k] - x[0]) / L);
    w *= w;
    num += (lower[k - 1] + upper[k - 1]) * std::cos(kPi * (x[k] - x[k - 1]) / L) * w;
    den += diag[(k - 1) * dstride] * w;
  }
  return std::fabs(num / den);
}

static double omega_of(double rho) {
  if (rho > 1.0) rho = 1.0;
  double t = 1.0 - rho * rho;
  if (t < 0.0) t = 0.0;
  return 2.0 / (1.0 + std::sqrt(t));
}

// Eigen-decomposition of a symmetric n x n matrix (row-major) by cyclic
// Jacobi rotations: on return a is diagonal (the eigenvalues) and the
// columns of q are the eigenvectors.
static void jacobi_eigen(std::vector<double>& a, std::vector<double>& q, int n) {
  q.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) q[(size_t)i * n + i] = 1.0;
  double scale = 0.0;
  for (double v : a) scale += v * v;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int r = p + 1; r < n; ++r) off += a[(size_t)p * n + r] * a[(size_t)p * n + r];
    if (off <= 1e-32 * scale) break;
    for (int p = 0; p < n; ++p)
      for (int r = p + 1; r < n; ++r) {
        const double apr = a[(size_t)p * n + r];
        if (apr == 0.0) continue;
        const double th = (a[(size_t)r * n + r] - a[(size_t)p * n + p]) / (2.0 * apr);
        const double t = (th >= 0.0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < n; ++k) {  // columns p, r
          const double x = a[(size_t)k * n + p], y = a[(size_t)k * n + r];
          a[(size_t)k * n + p] = c * x - sn * y;
          a[(size_t)k * n + r] = sn * x + c * y;
        }
        for (int k = 0; k < n; ++k) {  // rows p, r
          const double x = a[(size_t)p * n + k], y = a[(size_t)r * n + k];
          a[(size_t)p * n + k] = c * x - sn * y;
          a[(size_t)r * n + k] = sn * x + c * y;
        }
        for (int k = 0; k < n; ++k) {
          const double x = q[(size_t)k * n + p], y = q[(size_t)k * n + r];
          q[(size_t)k * n + p] = c * x - sn * y;
          q[(size_t)k * n + r] = sn * x + c * y;
        }
      }
  }
}

// Fast diagonalisation of the level operator of every mode.  The operator
// is L = A (x) I + diag(Rr) (x) B with A = tridiag(da, Ca, ua) along a and
// B = tridiag(db, Cb, ub) along b.  B = D^-1 S D with D diagonal and S
// symmetric; S = Q Lambda Q^T gives B = V Lambda V^-1 with V = D^-1 Q and
// V^-1 = Q^T D, so L u = f becomes, with w = f V^-T row by row, the
// tridiagonal systems (A + lambda_q diag(Rr)) x_q = w_q along a, one per
// eigenvalue, and u = x V^T.  Stores V, V^-1 and the Thomas factors of
// every (mode, q); checks the factors against the operator on random
// right-hand sides and leaves the tables empty if they miss 1e-10 (the
// coarsest level then falls back to red-black SOR).
void separable_factors(LevelTables& T, int M) {
  const int n1 = T.na, n2 = T.nb;
  T.sep_v.clear(); T.sep_vi.clear(); T.sep_cp.clear(); T.sep_id.clear();
  if (n2 > 128) return;  // the device row transforms take at most 128 columns
  for (int j = 0; j + 1 < n2; ++j)
    if (!(T.ub[j] > 0.0) || !(T.db[j + 1] > 0.0)) return;
  std::vector<double> V((size_t)M * n2 * n2), Vi((size_t)M * n2 * n2), CP((size_t)M * n1 * n2), ID((size_t)M * n1 * n2);
  std::vector<double> d(n2), S, Q, lam(n2);
  for (int p = 0; p < M; ++p) {
    const double* Ca = &T.Ca[(size_t)p * n1];
    const double* Cb = &T.Cb[(size_t)p * n2];
    d[0] = 1.0;
    for (int j = 0; j + 1 < n2; ++j) d[j + 1] = d[j] * std::sqrt(T.ub[j] / T.db[j + 1]);
    S.assign((size_t)n2 * n2, 0.0);
    for (int j = 0; j < n2; ++j) {
      S[(size_t)j * n2 + j] = Cb[j];
      if (j + 1 < n2) S[(size_t)j * n2 + j + 1] = S[(size_t)(j + 1) * n2 + j] = std::sqrt(T.ub[j] * T.db[j + 1]);
    }
    jacobi_eigen(S, Q, n2);
    for (int q = 0; q < n2; ++q) lam[q] = S[(size_t)q * n2 + q];
    // stored transposed, so that consecutive outputs of a row transform read
    // consecutive table entries: v[q][j] = V[j][q], vi[j][q] = V^-1[q][j]
    double* v = &V[(size_t)p * n2 * n2];
    double* vi = &Vi[(size_t)p * n2 * n2];
    for (int j = 0; j < n2; ++j)
      for (int q = 0; q < n2; ++q) {
        v[(size_t)q * n2 + j] = Q[(size_t)j * n2 + q] / d[j];
        vi[(size_t)j * n2 + q] = Q[(size_t)j * n2 + q] * d[j];
      }
    double* cp = &CP[(size_t)p * n1 * n2];
    double* id = &ID[(size_t)p * n1 * n2];
    for (int q = 0; q < n2; ++q) {
      double prev = 0.0;
      for (int i = 0; i < n1; ++i) {
        const double den = Ca[i] + lam[q] * T.Rr[i] - (i > 0 ? T.da[i] * prev : 0.0);
        if (!(std::fabs(den) > 0.0)) return;
        id[(size_t)i * n2 + q] = 1.0 / den;
        prev = T.ua[i] / den;
        cp[(size_t)i * n2 + q] = prev;
      }
    }
    // check: a random right-hand side solved and multiplied back
    std::vector<double> f((size_t)n1 * n2), w((size_t)n1 * n2), u((size_t)n1 * n2);
    unsigned long long st = 0x9E3779B97F4A7C15ull * (unsigned long long)(p + 1);
    for (double& x : f) {
      st = st * 6364136223846793005ull + 1442695040888963407ull;
      x = (double)(st >> 11) / 9007199254740992.0 - 0.5;
    }
    for (int i = 0; i < n1; ++i)
      for (int q = 0; q < n2; ++q) {
        double acc = 0.0;
        for (int j = 0; j < n2; ++j) acc += vi[(size_t)j * n2 + q] * f[(size_t)i * n2 + j];
        w[(size_t)i * n2 + q] = acc;
      }
    for (int q = 0; q < n2; ++q) {
      double prev = 0.0;
      for (int i = 0; i < n1; ++i) {
        prev = (w[(size_t)i * n2 + q] - (i > 0 ? T.da[i] * prev : 0.0)) * id[(size_t)i * n2 + q];
        w[(size_t)i * n2 + q] = prev;
      }
      for (int i = n1 - 2; i >= 0; --i) w[(size_t)i * n2 + q] -= cp[(size_t)i * n2 + q] * w[(size_t)(i + 1) * n2 + q];
    }
    for (int i = 0; i < n1; ++i)
      for (int j = 0; j < n2; ++j) {
        double acc = 0.0;
        for (int q = 0; q < n2; ++q) acc += v[(size_t)q * n2 + j] * w[(size_t)i * n2 + q];
        u[(size_t)i * n2 + j] = acc;
      }
    double r2 = 0.0, f2 = 0.0;
    for (int i = 0; i < n1; ++i)
      for (int j = 0; j < n2; ++j) {
        double Lu = (Ca[i] + T.Rr[i] * Cb[j]) * u[(size_t)i * n2 + j];
        if (i + 1 < n1) Lu += T.ua[i] * u[(size_t)(i + 1) * n2 + j];
        if (i > 0) Lu += T.da[i] * u[(size_t)(i - 1) * n2 + j];
        if (j + 1 < n2) Lu += T.Rr[i] * T.ub[j] * u[(size_t)i * n2 + j + 1];
        if (j > 0) Lu += T.Rr[i] * T.db[j] * u[(size_t)i * n2 + j - 1];
        const double r = Lu - f[(size_t)i * n2 + j];
        r2 += r * r;
        f2 += f[(size_t)i * n2 + j] * f[(size_t)i * n2 + j];
      }
    if (!(r2 <= 1e-20 * f2)) return;
  }
  T.sep_v.swap(V);
  T.sep_vi.swap(Vi);
  T.sep_cp.swap(CP);
  T.sep_id.swap(ID);
}

static double transfer_coord(const Spec& s, char which, double x) {
  return (which == 'a' && s.sph()) ? x * x : x;
}

Hierarchy build_hierarchy(const Spec& s, long a_lo, int na, long b_lo, int nb, const int edge[4],
                          const std::vector<int>& modes, bool main_grid, int max_coarse, bool exact_coarse) {
  Hierarchy h;
  h.spec = s;
  h.M = (int)modes.size();
  // level sizes: halve while the level has more than max_coarse cells (a
  // level that small is the coarsest and is solved exactly) -- but at least
  // once, so that there is a coarse-grid correction -- while both sides are
  // even, the smaller coarse side stays >= 2 and the coarse inner radial
  // ghost face stays at r > 0.
  if (max_coarse < 1) max_coarse = kMaxDirect;
  std::vector<std::pair<int, int>> sizes{{na, nb}};
  long stride = 1;
  while (true) {
    int ca = sizes.back().first, cb = sizes.back().second;
    if (ca * cb <= max_coarse && sizes.size() > 1) {
      h.stop = "the level is small enough";
      break;
    }
    if ((ca % 2) || (cb % 2)) {
      h.stop = "a side of the level is odd";
      break;
    }
    if (std::min(ca, cb) / 2 < 2) {
      h.stop = "halving would leave a side below 2 cells";
      break;
    }
    if (s.radial_face((double)((a_lo - 1) - 2 * stride)) <= 0.0) {
      h.stop = "the coarse inner radial ghost face would reach r <= 0";
      break;
    }
    sizes.push_back({ca / 2, cb / 2});
    stride *= 2;
  }
  (void)main_grid;
  int L = (int)sizes.size();
  h.lv.resize(L);
  for (int l = 0; l < L; ++l) {
    LevelTables& T = h.lv[l];
    long st = 1L << l;
    T.na = sizes[l].first;
    T.nb = sizes[l].second;
    for (int e = 0; e < 4; ++e) T.edge[e] = edge[e];
    T.A = make_axis(s, 'a', a_lo - 1, st, T.na);
    T.B = make_axis(s, 'b', b_lo - 1, st, T.nb);
    const Axis &A = T.A, &B = T.B;
    for (int e = 0; e < 4; ++e) T.dk[e] = 0.0;
    if (l > 0) {
      for (int ax = 0; ax < 2; ++ax) {
        const Axis& f0 = ax ? h.lv[0].B : h.lv[0].A;
        const Axis& c = ax ? B : A;
        double xg = f0.cent[0];
        T.dk[2 * ax] = -(xg - c.cent[0]) / (c.cent[1] - xg);
        xg = f0.cent[f0.n + 1];
        T.dk[2 * ax + 1] = -(c.cent[c.n + 1] - xg) / (xg - c.cent[c.n]);
      }
    }
    auto kap = [&](int e, int m) { return edge[e] == EDGE_DIRICHLET ? T.dk[e] : kappa(edge[e], m); };
    int n1 = T.na, n2 = T.nb;
    T.ua.resize(n1); T.da.resize(n1); T.Rr.resize(n1);
    T.ub.resize(n2); T.db.resize(n2);
    for (int i = 0; i < n1; ++i) {
      T.ua[i] = (i == n1 - 1) ? 0.0 : A.up[i + 1];
      T.da[i] = (i == 0) ? 0.0 : A.dn[i + 1];
      T.Rr[i] = s.sph() ? A.R[i + 1] : 1.0;
    }
    for (int j = 0; j < n2; ++j) {
      T.ub[j] = (j == n2 - 1) ? 0.0 : B.up[j + 1];
      T.db[j] = (j == 0) ? 0.0 : B.dn[j + 1];
    }
    int M = h.M;
    T.Ca.assign((size_t)M * n1, 0.0);
    T.Cb.assign((size_t)M * n2, 0.0);
    T.wr.assign((size_t)M * n2, 1.0);
    T.wb.assign((size_t)M * n1, 1.0);
    T.wc.assign(M, 1.0);
    for (int p = 0; p < M; ++p) {
      int m = modes[p];
      double s2 = mode_s2(s.n_phi, m);
      double* Ca = &T.Ca[(size_t)p * n1];
      double* Cb = &T.Cb[(size_t)p * n2];
      for (int i = 0; i < n1; ++i) {
        double dn = A.dn[i + 1];
        if (i == 0) dn = (edge[0] == EDGE_NEUMANN) ? 0.0 : dn * (1.0 - kap(0, m));
        Ca[i] = -(A.up[i + 1] + dn);
        if (i == n1 - 1) Ca[i] += kap(1, m) * A.up[i + 1];
        if (!s.sph()) Ca[i] -= s2 * A.P[i + 1];
      }
      for (int j = 0; j < n2; ++j) {
        Cb[j] = -(B.up[j + 1] + B.dn[j + 1]);
        if (j == 0) Cb[j] += kap(2, m) * B.dn[1];
        if (j == n2 - 1) Cb[j] += kap(3, m) * B.up[n2];
        if (s.sph()) Cb[j] -= s2 * B.P[j + 1];
      }
      // WKB omegas: radial line j (points i), polar line i (points j)
      std::vector<double> diag(n1), lo(n2), hi(n2), dg(n2);
      for (int j = 0; j < n2; ++j) {
        for (int i = 0; i < n1; ++i) diag[i] = Ca[i] + T.Rr[i] * Cb[j];
        T.wr[(size_t)p * n2 + j] = omega_of(wkb_radius(A.cent.data(), n1, T.da.data(), T.ua.data(), diag.data(), 1));
      }
      for (int i = 0; i < n1; ++i) {
        for (int j = 0; j < n2; ++j) {
          lo[j] = T.Rr[i] * T.db[j];
          hi[j] = T.Rr[i] * T.ub[j];
          dg[j] = Ca[i] + T.Rr[i] * Cb[j];
        }
        T.wb[(size_t)p * n1 + i] = omega_of(wkb_radius(B.cent.data(), n2, lo.data(), hi.data(), dg.data(), 1));
      }
      // 2D estimate (p = q = 1 term of Appendix A's 2D formula)
      double La = A.cent[n1 + 1] - A.cent[0], Lb = B.cent[n2 + 1] - B.cent[0];
      double num = 0.0, den = 0.0;
      for (int i = 0; i < n1; ++i) {
        double wa = std::sin(kPi * (A.cent[i + 1] - A.cent[0]) / La);
        wa *= wa;
        double ca = std::cos(kPi * (A.cent[i + 1] - A.cent[i]) / La);
        for (int j = 0; j < n2; ++j) {
          double wbv = std::sin(kPi * (B.cent[j + 1] - B.cent[0]) / Lb);
          wbv *= wbv;
          double cbv = std::cos(kPi * (B.cent[j + 1] - B.cent[j]) / Lb);
          double w = wa * wbv;
          num += ((T.ua[i] + T.da[i]) * ca + T.Rr[i] * (T.ub[j] + T.db[j]) * cbv) * w;
          den += (Ca[i] + T.Rr[i] * Cb[j]) * w;
        }
      }
      T.wc[p] = omega_of(std::fabs(num / den));
    }
    // normalised volume weights
    double sa = 0.0, sb = 0.0;
    T.va.resize(n1);
    T.vb.resize(n2);
    for (int i = 0; i < n1; ++i) sa += A.vol[i + 1];
    for (int j = 0; j < n2; ++j) sb += B.vol[j + 1];
    for (int i = 0; i < n1; ++i) T.va[i] = A.vol[i + 1] / sa;
    for (int j = 0; j < n2; ++j) T.vb[j] = B.vol[j + 1] / sb;
  }
  // exact solve of the coarsest level by fast diagonalisation
  if (exact_coarse) {
    LevelTables& T = h.lv[L - 1];
    separable_factors(T, h.M);
  }
  // transfers between consecutive levels (bilinear in (r^2, theta) or (R, z);
  // restriction: the printed area weights read as opposite-corner weights)
  for (int l = 0; l + 1 < L; ++l) {
    LevelTables &F = h.lv[l], &C = h.lv[l + 1];
    for (int ax = 0; ax < 2; ++ax) {
      const Axis& fa = ax ? F.B : F.A;
      const Axis& caa = ax ? C.B : C.A;
      char which = ax ? 'b' : 'a';
      int nc = caa.n, nf = fa.n;
      std::vector<double>& rw = ax ? F.rwb : F.rwa;
      rw.resize(2 * nc);
      for (int I = 1; I <= nc; ++I) {
        double xl = transfer_coord(s, which, fa.cent[2 * I - 1]);
        double xh = transfer_coord(s, which, fa.cent[2 * I]);
        double X = transfer_coord(s, which, caa.cent[I]);
        rw[2 * (I - 1) + 0] = std::fabs(xh - X) / std::fabs(xh - xl);
        rw[2 * (I - 1) + 1] = std::fabs(X - xl) / std::fabs(xh - xl);
      }
      for (int par = 0; par < (ax ? 2 : 1); ++par) {
        const int elo = ax ? 2 : 0, ehi = ax ? 3 : 1;
        double k_lo = edge[elo] == EDGE_DIRICHLET ? C.dk[elo] : kappa(edge[elo], par);
        double k_hi = edge[ehi] == EDGE_DIRICHLET ? C.dk[ehi] : kappa(edge[ehi], par);
        std::vector<int> i0(nf), i1(nf);
        std::vector<double> w0(nf), w1(nf);
        for (int k = 1; k <= nf; ++k) {
          int I = (k + 1) / 2;
          int c0 = (k % 2) ? I - 1 : I;
          int c1 = c0 + 1;
          double x0 = transfer_coord(s, which, caa.cent[c0]);
          double x1 = transfer_coord(s, which, caa.cent[c1]);
          double x = transfer_coord(s, which, fa.cent[k]);
          double a0 = std::fabs(x1 - x) / std::fabs(x1 - x0);
          double a1 = std::fabs(x - x0) / std::fabs(x1 - x0);
          int j0 = c0 - 1, j1 = c1 - 1;
          if (c0 == 0) { j0 = 0; a0 *= k_lo; }
          if (c1 == nc + 1) { j1 = nc - 1; a1 *= k_hi; }
          i0[k - 1] = j0; i1[k - 1] = j1; w0[k - 1] = a0; w1[k - 1] = a1;
        }
        if (ax == 0) {
          F.pa_i0 = i0; F.pa_i1 = i1; F.pa_w0 = w0; F.pa_w1 = w1;
        } else {
          F.pb_i0[par] = i0; F.pb_i1[par] = i1; F.pb_w0[par] = w0; F.pb_w1[par] = w1;
        }
      }
    }
  }
  return h;
}

GhostSet make_ghosts(const Spec& s) {
  GhostSet g;
  Axis A = make_axis(s, 'a', 0, 1, s.n_a);
  Axis B = make_axis(s, 'b', 0, 1, s.n_b);
  auto add = [&](int i, int j, int e, double cout, double cin) {
    g.gi.push_back(i);
    g.gj.push_back(j);
    g.edge.push_back(e);
    g.a.push_back(A.cent[i]);
    g.b.push_back(B.cent[j]);
    g.dv3.push_back(A.vol[i] * B.vol[j] * s.dphi());
    g.coup_out.push_back(cout);
    g.coup_in.push_back(cin);
    int ia = std::min(std::max(i, 1), s.n_a) - 1;
    int jb = std::min(std::max(j, 1), s.n_b) - 1;
    g.adj.push_back(ia * s.n_b + jb);
  };
  for (int j = 1; j <= s.n_b; ++j) add(0, j, 0, A.up[0], A.dn[1]);
  for (int j = 1; j <= s.n_b; ++j) add(s.n_a + 1, j, 1, A.dn[s.n_a + 1], A.up[s.n_a]);
  if (!s.pole_lo())
    for (int i = 1; i <= s.n_a; ++i) {
      double R = s.sph() ? A.R[i] : 1.0;
      add(i, 0, 2, R * B.up[0], R * B.dn[1]);
    }
  if (!s.pole_hi())
    for (int i = 1; i <= s.n_a; ++i) {
      double R = s.sph() ? A.R[i] : 1.0;
      add(i, s.n_b + 1, 3, R * B.dn[s.n_b + 1], R * B.up[s.n_b]);
    }
  g.n = (int)g.gi.size();
  return g;
}

}  // namespace smg
