// C ABI of the smg library (include/smg.h): plan creation and validation,
// workspace layout, device setup (table upload, DGF construction), the
// batched multigrid driver and the seven-step solve of Sec. 5.1.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "dgf_dev.h"
#include "smg_internal.h"

using namespace smg;

static thread_local std::string g_err;

static smg_status fail(smg_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIPCHK(expr)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return fail(SMG_EHIP, strprintf("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                                      __FILE__, __LINE__));                                 \
  } while (0)

#define STCHK(expr)                  \
  do {                               \
    smg_status s_ = (expr);          \
    if (s_ != SMG_OK) return s_;     \
  } while (0)

namespace {

constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr size_t kAlign = 256;
constexpr int kNormBlocks = 64;
constexpr double kFloor = 1e-6;          // stopping-rule floor factor
constexpr double kCoarseRtol = 1e-10;    // coarsest red-black SOR
constexpr int kCoarseSweeps = 1000;
constexpr int kMaxCoarseCells = 1024;
constexpr int kMaxLine = 512;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Packs host tables into one device blob; offsets are 256-byte aligned.
struct Blob {
  std::vector<char> bytes;
  size_t add(const void* p, size_t n) {
    size_t off = align_up(bytes.size());
    bytes.resize(off + (n ? n : 1));
    if (n) std::memcpy(bytes.data() + off, p, n);
    return off;
  }
  template <class T>
  size_t add(const std::vector<T>& v) {
    return add(v.data(), v.size() * sizeof(T));
  }
};

// Offsets of one level's tables inside the blob.
struct LevelOff {
  size_t ua, da, Rr, ub, db, Ca, Cb, wr, wb, wc, va, vb, rwa, rwb, pa_i0, pa_i1, pa_w0, pa_w1, pb_i0, pb_i1,
      pb_w0, pb_w1, cinv;
  bool has_cinv;
};

LevelOff pack_level(Blob& B, const LevelTables& T) {
  LevelOff o{};
  o.ua = B.add(T.ua); o.da = B.add(T.da); o.Rr = B.add(T.Rr); o.ub = B.add(T.ub); o.db = B.add(T.db);
  o.Ca = B.add(T.Ca); o.Cb = B.add(T.Cb); o.wr = B.add(T.wr); o.wb = B.add(T.wb); o.wc = B.add(T.wc);
  o.va = B.add(T.va); o.vb = B.add(T.vb);
  o.rwa = B.add(T.rwa); o.rwb = B.add(T.rwb);
  o.pa_i0 = B.add(T.pa_i0); o.pa_i1 = B.add(T.pa_i1); o.pa_w0 = B.add(T.pa_w0); o.pa_w1 = B.add(T.pa_w1);
  std::vector<int> i0, i1;
  std::vector<double> w0, w1;
  for (int par = 0; par < 2; ++par) {
    i0.insert(i0.end(), T.pb_i0[par].begin(), T.pb_i0[par].end());
    i1.insert(i1.end(), T.pb_i1[par].begin(), T.pb_i1[par].end());
    w0.insert(w0.end(), T.pb_w0[par].begin(), T.pb_w0[par].end());
    w1.insert(w1.end(), T.pb_w1[par].begin(), T.pb_w1[par].end());
  }
  o.pb_i0 = B.add(i0); o.pb_i1 = B.add(i1); o.pb_w0 = B.add(w0); o.pb_w1 = B.add(w1);
  o.has_cinv = !T.cinv.empty();
  o.cinv = o.has_cinv ? B.add(T.cinv) : 0;
  return o;
}

LevelDev level_view(const char* base, const LevelOff& o, const LevelTables& T, int M) {
  LevelDev L{};
  L.na = T.na; L.nb = T.nb; L.M = M;
  auto d = [&](size_t off) { return reinterpret_cast<const double*>(base + off); };
  auto i = [&](size_t off) { return reinterpret_cast<const int*>(base + off); };
  L.ua = d(o.ua); L.da = d(o.da); L.Rr = d(o.Rr); L.ub = d(o.ub); L.db = d(o.db);
  L.Ca = d(o.Ca); L.Cb = d(o.Cb); L.wr = d(o.wr); L.wb = d(o.wb); L.wc = d(o.wc);
  L.va = d(o.va); L.vb = d(o.vb); L.rwa = d(o.rwa); L.rwb = d(o.rwb);
  L.pa_i0 = i(o.pa_i0); L.pa_i1 = i(o.pa_i1); L.pa_w0 = d(o.pa_w0); L.pa_w1 = d(o.pa_w1);
  L.pb_i0 = i(o.pb_i0); L.pb_i1 = i(o.pb_i1); L.pb_w0 = d(o.pb_w0); L.pb_w1 = d(o.pb_w1);
  L.cinv = o.has_cinv ? d(o.cinv) : nullptr;
  return L;
}

// Fields of one multigrid run: level 0 is supplied per call, coarser levels
// hold `cap` planes each.
struct MGFields {
  std::vector<LevelDev> L;
  std::vector<double2*> u, f;  // index 0 unused
  bool exact = false;          // exact (Thomas) line relaxation
  bool fp32 = false;           // mixed form: FP32 correction cycles
  std::vector<float2*> u32, f32;  // FP32 correction / right-hand side per level (mixed form)
  int lds_first = 0;           // first level of the in-LDS coarse cycle
  LdsLevels lds{};
};

constexpr size_t kLdsCycleMax = 63 * 1024;  // leaves room for the static reduction buffer

// Choose the deepest run of levels (ending at the coarsest) that one block
// can hold in LDS, starting as fine as possible.
void plan_lds(MGFields& F) {
  const int L = (int)F.L.size();
  for (int first = 0; first < L; ++first) {
    if (L - first > kMaxLdsLevels) continue;
    LdsLevels LL{};
    LL.n = L - first;
    int words = 0;
    for (int l = first; l < L; ++l) {
      LL.L[l - first] = F.L[l];
      words += (F.L[l].na + 2) * (F.L[l].nb + 2) + F.L[l].na * F.L[l].nb;
    }
    LL.words = words;
    LL.scratch = smgk::lds_cycle_scratch(LL, F.exact);
    if (smgk::lds_cycle_bytes(LL, F.fp32) <= kLdsCycleMax) {
      F.lds_first = first;
      F.lds = LL;
      return;
    }
  }
  F.lds_first = L - 1;
}

}  // namespace

struct smg_plan {
  Spec spec{};
  smg_opts opts{};
  Hierarchy H;
  GhostSet gh;
  int M = 0, n_g = 0;
  // boundary cells receiving ghost data (solve 2)
  std::vector<int> ap_cell, ap_g0, ap_g1;
  std::vector<double> ap_c0, ap_c1;
  // host tables packed for upload
  Blob blob;
  std::vector<LevelOff> loff;
  size_t o_tw = 0, o_adj = 0, o_cout = 0, o_apc = 0, o_apg0 = 0, o_apg1 = 0, o_apc0 = 0, o_apc1 = 0;
  // workspace layout (byte offsets)
  size_t w_blob = 0, w_dgf = 0, w_psi = 0, w_phi = 0, w_f = 0, w_sigma = 0, w_theta = 0, w_partial = 0,
         w_norm = 0, w_slot = 0, w_mode = 0, w_total = 0;
  std::vector<size_t> w_u, w_fl, w_u32, w_f32;
  // bound workspace
  char* ws = nullptr;
  bool ready = false;
  bool have_prev = false;
  double dgf_resid = 0.0;  // worst relative residual of the DGF solves
  MGFields mg;
  // per-launch event timing (smg_profile_begin / smg_profile_end)
  struct ProfRec { int cls, ev0, ev1; double bytes; };
  mutable bool prof_on = false;
  mutable std::vector<hipEvent_t> prof_pool;
  mutable size_t prof_used = 0;
  mutable std::vector<ProfRec> prof_log;
  // pinned host staging
  int* h_slot = nullptr;
  int* h_mode = nullptr;
  double* h_norm = nullptr;
  ~smg_plan() {
    for (hipEvent_t e : prof_pool) (void)hipEventDestroy(e);
    if (h_slot) (void)hipHostFree(h_slot);
    if (h_mode) (void)hipHostFree(h_mode);
    if (h_norm) (void)hipHostFree(h_norm);
  }
  double2* dptr(size_t off) const { return reinterpret_cast<double2*>(ws + off); }
};

// ----------------------------------------------------------------------------
// validation and plan creation
// ----------------------------------------------------------------------------
static bool is_2p3q(int n) {
  if (n < 1) return false;
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  return n == 1;
}

static smg_status validate(const smg_grid& g, const smg_opts& o) {
  if (g.geometry != SMG_SPHERICAL && g.geometry != SMG_CYLINDRICAL) return fail(SMG_EINVAL, "geometry must be SMG_SPHERICAL or SMG_CYLINDRICAL");
  if (g.radial != SMG_RADIAL_UNIFORM && g.radial != SMG_RADIAL_LOG) return fail(SMG_EINVAL, "radial must be SMG_RADIAL_UNIFORM or SMG_RADIAL_LOG");
  if (g.n_a < 4 || g.n_b < 4 || (g.n_a & 1) || (g.n_b & 1)) return fail(SMG_EINVAL, "n_a and n_b must be even and >= 4");
  if (g.n_a > kMaxLine || g.n_b > kMaxLine) return fail(SMG_EINVAL, strprintf("n_a and n_b must be <= %d", kMaxLine));
  if (g.n_phi < 4 || (g.n_phi & 1) || !is_2p3q(g.n_phi / 2) || g.n_phi / 2 > 1024)
    return fail(SMG_EINVAL, "n_phi must be even, >= 4, with n_phi/2 = 2^p 3^q <= 1024");
  if (!(g.a_min > 0.0) || !(g.a_max > g.a_min) || !std::isfinite(g.a_max)) return fail(SMG_EINVAL, "need 0 < a_min < a_max");
  if (!(g.b_max > g.b_min) || !std::isfinite(g.b_min) || !std::isfinite(g.b_max)) return fail(SMG_EINVAL, "need b_min < b_max");
  if (g.geometry == SMG_SPHERICAL && (g.b_min < 0.0 || g.b_max > kPi + 1e-12)) return fail(SMG_EINVAL, "theta range must lie in [0, pi]");
  if (!(g.G > 0.0)) return fail(SMG_EINVAL, "G must be > 0");
  if (g.radial == SMG_RADIAL_UNIFORM && g.a_min - (g.a_max - g.a_min) / g.n_a <= 0.0)
    return fail(SMG_EINVAL, "uniform radial grid: the inner ghost cell reaches r <= 0");
  if (o.precision != SMG_FP64 && o.precision != SMG_MIXED) return fail(SMG_EINVAL, "precision must be SMG_FP64 or SMG_MIXED");
  if (o.nu_pre < 0 || o.nu_post < 0 || o.nu_pre + o.nu_post < 1 || o.n_sor < 1 || o.max_cycles < 1)
    return fail(SMG_EINVAL, "need nu_pre + nu_post >= 1, n_sor >= 1, max_cycles >= 1");
  if (o.n_pad < 2 || o.n_pad > 24) return fail(SMG_EINVAL, "n_pad must be in [2, 24]");
  if (o.dgf_method < SMG_DGF_AUTO || o.dgf_method > SMG_DGF_EXTENDED) return fail(SMG_EINVAL, "bad dgf_method");
  if (o.line_solver != SMG_LINE_SOR && o.line_solver != SMG_LINE_EXACT) return fail(SMG_EINVAL, "bad line_solver");
  return SMG_OK;
}

static int dgf_method_of(const smg_plan& p) {
  if (p.opts.dgf_method != SMG_DGF_AUTO) return p.opts.dgf_method;
  return p.spec.radial == SMG_RADIAL_LOG ? SMG_DGF_EXTENDED : SMG_DGF_AUX;
}

extern "C" smg_status smg_plan_create(const smg_grid* grid, const smg_opts* opts_in, smg_plan** out) {
  if (!grid || !out) return fail(SMG_EINVAL, "grid and out must not be NULL");
  *out = nullptr;
  smg_opts o{};
  if (opts_in) o = *opts_in;
  if (o.nu_pre == 0 && o.nu_post == 0) { o.nu_pre = 2; o.nu_post = 2; }
  if (o.n_sor == 0) o.n_sor = 2;
  if (o.max_cycles == 0) o.max_cycles = 60;
  if (o.n_pad == 0) o.n_pad = 16;
  if (o.dgf_tol == 0.0) o.dgf_tol = 1e-13;
  STCHK(validate(*grid, o));
  std::unique_ptr<smg_plan> p(new (std::nothrow) smg_plan());
  if (!p) return fail(SMG_EINVAL, "out of host memory");
  Spec& s = p->spec;
  s.geometry = grid->geometry; s.radial = grid->radial;
  s.n_a = grid->n_a; s.n_b = grid->n_b; s.n_phi = grid->n_phi;
  s.a_min = grid->a_min; s.a_max = grid->a_max; s.b_min = grid->b_min; s.b_max = grid->b_max; s.G = grid->G;
  p->opts = o;
  p->M = s.n_modes();
  int edge[4] = {EDGE_DIRICHLET, EDGE_DIRICHLET, s.pole_lo() ? EDGE_POLE : EDGE_DIRICHLET,
                 s.pole_hi() ? EDGE_POLE : EDGE_DIRICHLET};
  std::vector<int> modes(p->M);
  for (int m = 0; m < p->M; ++m) modes[m] = m;
  p->H = build_hierarchy(s, 1, s.n_a, 1, s.n_b, edge, modes, true);
  const LevelTables& Lc = p->H.lv.back();
  if (Lc.na * Lc.nb > kMaxCoarseCells)
    return fail(SMG_EINVAL, strprintf("grid coarsens only to %dx%d (> %d cells): the radial ghost face reaches r <= 0",
                                      Lc.na, Lc.nb, kMaxCoarseCells));
  p->gh = make_ghosts(s);
  p->n_g = p->gh.n;
  if (p->n_g > 4096) return fail(SMG_EINVAL, "too many boundary ghost cells (> 4096)");
  // DGF geometry checks
  int meth = dgf_method_of(*p);
  if (meth == SMG_DGF_EXTENDED) {
    if (s.n_a <= o.n_pad) return fail(SMG_EINVAL, "extended DGF domain needs n_a > n_pad");
    if (2 * s.n_a > kMaxLine) return fail(SMG_EINVAL, "extended DGF domain: 2 n_a exceeds the line limit");
    if (!(s.pole_lo() && s.pole_hi()) && 2 * s.n_b > kMaxLine) return fail(SMG_EINVAL, "extended DGF domain: 2 n_b exceeds the line limit");
    if (s.radial == SMG_RADIAL_UNIFORM && s.radial_face(-(double)(s.n_a - o.n_pad) - 1.0) <= 0.0)
      return fail(SMG_EINVAL, "extended DGF domain reaches r <= 0 on this uniform grid; use the auxiliary grid");
    if (s.sph() && !(s.pole_lo() && s.pole_hi())) {
      long ext = s.n_b / 2;
      if ((!s.pole_lo() && s.b_face(-ext - 1) < 0.0) || (!s.pole_hi() && s.b_face(s.n_b + ext + 1) > kPi))
        return fail(SMG_EINVAL, "extended DGF domain crosses a pole away from the grid edge");
    }
  }
  // boundary cells of solve 2 (each interior cell gathers its adjacent ghosts)
  {
    std::vector<int> first(s.n_a * s.n_b, -1), second(s.n_a * s.n_b, -1);
    for (int g = 0; g < p->n_g; ++g) {
      int c = p->gh.adj[g];
      if (first[c] < 0) first[c] = g; else second[c] = g;
    }
    for (int c = 0; c < s.n_a * s.n_b; ++c) {
      if (first[c] < 0) continue;
      p->ap_cell.push_back(c);
      p->ap_g0.push_back(first[c]);
      p->ap_c0.push_back(p->gh.coup_in[first[c]]);
      p->ap_g1.push_back(second[c]);
      p->ap_c1.push_back(second[c] >= 0 ? p->gh.coup_in[second[c]] : 0.0);
    }
  }
  // pack tables
  for (const LevelTables& T : p->H.lv) p->loff.push_back(pack_level(p->blob, T));
  {
    int n = s.n_phi / 2;
    std::vector<double2> tw(2 * n + 1);
    for (int k = 0; k < n; ++k) tw[k] = make_double2(std::cos(2.0 * kPi * k / n), -std::sin(2.0 * kPi * k / n));
    for (int m = 0; m <= n; ++m)
      tw[n + m] = make_double2(std::cos(2.0 * kPi * m / s.n_phi), -std::sin(2.0 * kPi * m / s.n_phi));
    p->o_tw = p->blob.add(tw);
  }
  p->o_adj = p->blob.add(p->gh.adj);
  p->o_cout = p->blob.add(p->gh.coup_out);
  p->o_apc = p->blob.add(p->ap_cell);
  p->o_apg0 = p->blob.add(p->ap_g0);
  p->o_apg1 = p->blob.add(p->ap_g1);
  p->o_apc0 = p->blob.add(p->ap_c0);
  p->o_apc1 = p->blob.add(p->ap_c1);
  // workspace layout
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o2 = off; off = align_up(off + bytes); return o2; };
  const size_t plane = (size_t)s.n_a * s.n_b;
  const int M = p->M;
  p->w_blob = take(p->blob.bytes.size());
  p->w_dgf = take(sizeof(double) * (size_t)M * p->n_g * p->n_g);
  p->w_psi = take(sizeof(double2) * M * plane);
  p->w_phi = take(sizeof(double2) * M * plane);
  p->w_f = take(sizeof(double2) * M * plane);
  p->w_sigma = take(sizeof(double2) * (size_t)M * p->n_g);
  p->w_theta = take(sizeof(double2) * (size_t)M * p->n_g);
  p->w_partial = take(sizeof(double) * (size_t)M * kNormBlocks);
  p->w_norm = take(sizeof(double) * M);
  p->w_slot = take(sizeof(int) * M);
  p->w_mode = take(sizeof(int) * M);
  p->w_u.assign(p->H.lv.size(), 0);
  p->w_fl.assign(p->H.lv.size(), 0);
  for (size_t l = 1; l < p->H.lv.size(); ++l) {
    size_t pl = (size_t)p->H.lv[l].na * p->H.lv[l].nb;
    p->w_u[l] = take(sizeof(double2) * M * pl);
    p->w_fl[l] = take(sizeof(double2) * M * pl);
  }
  if (o.precision == SMG_MIXED) {
    p->w_u32.assign(p->H.lv.size(), 0);
    p->w_f32.assign(p->H.lv.size(), 0);
    for (size_t l = 0; l < p->H.lv.size(); ++l) {
      size_t pl = (size_t)p->H.lv[l].na * p->H.lv[l].nb;
      p->w_u32[l] = take(sizeof(float2) * M * pl);
      p->w_f32[l] = take(sizeof(float2) * M * pl);
    }
  }
  p->w_total = off;
  *out = p.release();
  g_err.clear();
  return SMG_OK;
}

extern "C" size_t smg_workspace_bytes(const smg_plan* p) { return p ? p->w_total : 0; }

extern "C" smg_status smg_plan_destroy(smg_plan* p) {
  delete p;
  return SMG_OK;
}

extern "C" const char* smg_last_error(void) { return g_err.c_str(); }

extern "C" smg_status smg_plan_geometry(const smg_plan* p, double* a, double* b, double* phi, double* dv) {
  if (!p) return fail(SMG_EINVAL, "NULL plan");
  const Spec& s = p->spec;
  const LevelTables& T = p->H.lv[0];
  if (a) for (int i = 0; i < s.n_a; ++i) a[i] = T.A.cent[i + 1];
  if (b) for (int j = 0; j < s.n_b; ++j) b[j] = T.B.cent[j + 1];
  if (phi) for (int k = 0; k < s.n_phi; ++k) phi[k] = (k + 0.5) * s.dphi();
  if (dv)
    for (int i = 0; i < s.n_a; ++i)
      for (int j = 0; j < s.n_b; ++j) dv[(size_t)i * s.n_b + j] = T.A.vol[i + 1] * T.B.vol[j + 1] * s.dphi();
  return SMG_OK;
}

extern "C" smg_status smg_plan_shape(const smg_plan* p, int* n_levels, int* n_ghost, int* lna, int* lnb) {
  if (!p) return fail(SMG_EINVAL, "NULL plan");
  if (n_levels) *n_levels = (int)p->H.lv.size();
  if (n_ghost) *n_ghost = p->n_g;
  for (size_t l = 0; l < p->H.lv.size() && l < 16; ++l) {
    if (lna) lna[l] = p->H.lv[l].na;
    if (lnb) lnb[l] = p->H.lv[l].nb;
  }
  return SMG_OK;
}

// ----------------------------------------------------------------------------
// per-launch timing
// ----------------------------------------------------------------------------
enum KernelClass {
  K_FFT_R2C, K_FFT_C2R, K_SMOOTH_RADIAL0, K_SMOOTH_POLAR0, K_SMOOTH_COARSE, K_RESTRICT, K_PROLONG, K_COARSE,
  K_NORM, K_SCREEN, K_CONV, K_APPLY, K_ACCUM, K_COUNT
};
static const char* kKernelNames[K_COUNT] = {
  "fft_r2c", "fft_c2r", "smooth_radial_lines_l0", "smooth_polar_lines_l0", "smooth_coarser_levels",
  "residual_restrict", "prolong_add", "lds_coarse_cycle", "defect_norm", "james_screen", "james_conv", "james_apply",
  "accumulate_fp64"};

static int prof_mark(const smg_plan& p, hipStream_t st) {
  if (!p.prof_on) return -1;
  if (p.prof_used == p.prof_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return -1;
    p.prof_pool.push_back(e);
  }
  if (hipEventRecord(p.prof_pool[p.prof_used], st) != hipSuccess) return -1;
  return (int)p.prof_used++;
}

static void prof_close(const smg_plan& p, int cls, int ev0, double bytes, hipStream_t st) {
  if (ev0 < 0) return;
  int ev1 = prof_mark(p, st);
  if (ev1 >= 0) p.prof_log.push_back({cls, ev0, ev1, bytes});
}

// ----------------------------------------------------------------------------
// multigrid driver
// ----------------------------------------------------------------------------
static smg_status vcycle(const smg_plan& p, const MGFields& F, const Batch& b, double2* u0, const double2* f0,
                         hipStream_t st) {
  const int L = (int)F.L.size();
  std::vector<double2*> u(L);
  std::vector<const double2*> f(L);
  u[0] = u0;
  f[0] = f0;
  for (int l = 1; l < L; ++l) { u[l] = F.u[l]; f[l] = F.f[l]; }
  auto cells = [&](int l) { return (double)b.n * F.L[l].na * F.L[l].nb; };
  auto smooth = [&](int l) -> smg_status {
    for (int dir = 0; dir < 2; ++dir) {
      int ev = prof_mark(p, st);
      HIPCHK(smgk::mg_smooth_dir(F.L[l], b, u[l], f[l], p.opts.n_sor, F.exact, dir, st));
      prof_close(p, l == 0 ? (dir == 0 ? K_SMOOTH_RADIAL0 : K_SMOOTH_POLAR0) : K_SMOOTH_COARSE, ev,
                 48.0 * cells(l), st);
    }
    return SMG_OK;
  };
  const int first = F.lds_first;
  for (int l = 0; l < first; ++l) {
    for (int k = 0; k < p.opts.nu_pre; ++k) STCHK(smooth(l));
    int ev = prof_mark(p, st);
    HIPCHK(smgk::mg_restrict_residual(F.L[l], F.L[l + 1], b, u[l], f[l], F.f[l + 1], F.u[l + 1], st));
    prof_close(p, K_RESTRICT, ev, 40.0 * cells(l), st);
  }
  {
    int ev = prof_mark(p, st);
    HIPCHK(smgk::mg_lds_cycle(F.lds, b, f[first], u[first], first == 0, p.opts.nu_pre, p.opts.nu_post, p.opts.n_sor,
                              F.exact, kCoarseRtol, kCoarseSweeps, st));
    prof_close(p, K_COARSE, ev, 32.0 * cells(first), st);
  }
  for (int l = first - 1; l >= 0; --l) {
    int ev = prof_mark(p, st);
    HIPCHK(smgk::mg_prolong_add(F.L[l], F.L[l + 1], b, u[l], u[l + 1], st));
    prof_close(p, K_PROLONG, ev, 36.0 * cells(l), st);
    for (int k = 0; k < p.opts.nu_post; ++k) STCHK(smooth(l));
  }
  return SMG_OK;
}

// One FP32 correction V-cycle of the mixed form: solves L e = r on level 0
// (F.u32[0] = e, zero on entry; F.f32[0] = r) with FP32 smoothing and
// transfers and the FP64 coarsest solve.
static smg_status vcycle32(const smg_plan& p, const MGFields& F, const Batch& b, hipStream_t st) {
  const int L = (int)F.L.size();
  auto cells = [&](int l) { return (double)b.n * F.L[l].na * F.L[l].nb; };
  auto smooth = [&](int l) -> smg_status {
    for (int dir = 0; dir < 2; ++dir) {
      int ev = prof_mark(p, st);
      HIPCHK(smgk::mg_smooth_dir32(F.L[l], b, F.u32[l], F.f32[l], p.opts.n_sor, F.exact, dir, st));
      prof_close(p, l == 0 ? (dir == 0 ? K_SMOOTH_RADIAL0 : K_SMOOTH_POLAR0) : K_SMOOTH_COARSE, ev,
                 24.0 * cells(l), st);
    }
    return SMG_OK;
  };
  const int first = F.lds_first;
  for (int l = 0; l < first; ++l) {
    for (int k = 0; k < p.opts.nu_pre; ++k) STCHK(smooth(l));
    int ev = prof_mark(p, st);
    HIPCHK(smgk::mg_restrict_residual32(F.L[l], F.L[l + 1], b, F.u32[l], F.f32[l], F.f32[l + 1], F.u32[l + 1], st));
    prof_close(p, K_RESTRICT, ev, 20.0 * cells(l), st);
  }
  {
    int ev = prof_mark(p, st);
    HIPCHK(smgk::mg_lds_cycle32(F.lds, b, F.f32[first], F.u32[first], first == 0, p.opts.nu_pre, p.opts.nu_post,
                                p.opts.n_sor, F.exact, kCoarseRtol, kCoarseSweeps, st));
    prof_close(p, K_COARSE, ev, 16.0 * cells(first), st);
  }
  for (int l = first - 1; l >= 0; --l) {
    int ev = prof_mark(p, st);
    HIPCHK(smgk::mg_prolong_add32(F.L[l], F.L[l + 1], b, F.u32[l], F.u32[l + 1], st));
    prof_close(p, K_PROLONG, ev, 18.0 * cells(l), st);
    for (int k = 0; k < p.opts.nu_post; ++k) STCHK(smooth(l));
  }
  (void)L;
  return SMG_OK;
}

// Iterate V-cycles on planes 0..n-1 (slot p, mode modes[p]) until each meets
// ||D|| <= tol * max(||D_0||, floor_factor * max ||D_0||).  d_slot/d_mode
// are device int arrays of capacity n; partial/norm device scratch.
struct SolveOut {
  std::vector<int> cycles;
  std::vector<double> resid;
  bool converged = true;
};

static smg_status mg_solve_planes(const smg_plan& p, const MGFields& F, int n, const int* modes, double2* u0,
                                  const double2* f0, double tol, double floor_factor, bool warm, int max_cycles,
                                  int* d_slot, int* d_mode, int* h_slot, int* h_mode, double* d_partial,
                                  double* d_norm, double* h_norm, hipStream_t st, SolveOut& out) {
  const LevelDev& L0 = F.L[0];
  const size_t plane = (size_t)L0.na * L0.nb;
  out.cycles.assign(n, 0);
  out.resid.assign(n, 0.0);
  out.converged = true;
  if (n == 0) return SMG_OK;
  if (!warm) HIPCHK(smgk::fill_zero(u0, (size_t)n * plane, st));
  for (int q = 0; q < n; ++q) { h_slot[q] = q; h_mode[q] = modes[q]; }
  HIPCHK(hipMemcpyAsync(d_slot, h_slot, sizeof(int) * n, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(d_mode, h_mode, sizeof(int) * n, hipMemcpyHostToDevice, st));
  Batch all{n, d_slot, d_mode};
  float2* r32 = F.fp32 ? F.f32[0] : nullptr;
  float2* e32 = F.fp32 ? F.u32[0] : nullptr;
  HIPCHK(smgk::mg_norms(L0, all, nullptr, f0, d_partial, d_norm, st, r32, e32));
  HIPCHK(hipMemcpyAsync(h_norm, d_norm, sizeof(double) * n, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  std::vector<double> d0(h_norm, h_norm + n), cur(n), thr(n);
  double dmax = 0.0;
  for (double v : d0) dmax = std::max(dmax, v);
  for (int q = 0; q < n; ++q) thr[q] = tol * std::max(d0[q], floor_factor * dmax);
  if (warm) {
    HIPCHK(smgk::mg_norms(L0, all, u0, f0, d_partial, d_norm, st, r32, e32));
    HIPCHK(hipMemcpyAsync(h_norm, d_norm, sizeof(double) * n, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    cur.assign(h_norm, h_norm + n);
  } else {
    cur = d0;
  }
  std::vector<int> active;
  for (int q = 0; q < n; ++q)
    if (cur[q] > thr[q]) active.push_back(q);
  while (!active.empty()) {
    const int na = (int)active.size();
    for (int k = 0; k < na; ++k) { h_slot[k] = active[k]; h_mode[k] = modes[active[k]]; }
    HIPCHK(hipMemcpyAsync(d_slot, h_slot, sizeof(int) * na, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d_mode, h_mode, sizeof(int) * na, hipMemcpyHostToDevice, st));
    Batch b{na, d_slot, d_mode};
    if (F.fp32) {
      // iterative refinement: FP32 correction cycle, FP64 accumulation, FP64
      // residual (stored rounded to FP32 for the next correction)
      STCHK(vcycle32(p, F, b, st));
      int ev = prof_mark(p, st);
      HIPCHK(smgk::mg_accumulate(L0, b, u0, e32, st));
      prof_close(p, K_ACCUM, ev, 40.0 * na * plane, st);
    } else {
      STCHK(vcycle(p, F, b, u0, f0, st));
    }
    int ev = prof_mark(p, st);
    HIPCHK(smgk::mg_norms(L0, b, u0, f0, d_partial, d_norm, st, r32, e32));
    prof_close(p, K_NORM, ev, (F.fp32 ? 48.0 : 32.0) * na * plane, st);
    HIPCHK(hipMemcpyAsync(h_norm, d_norm, sizeof(double) * na, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    std::vector<int> next;
    for (int k = 0; k < na; ++k) {
      const int q = active[k];
      cur[q] = h_norm[k];
      out.cycles[q] += 1;
      if (!(cur[q] <= thr[q]) && out.cycles[q] < max_cycles) next.push_back(q);
    }
    active.swap(next);
  }
  for (int q = 0; q < n; ++q) {
    const double den = std::max(d0[q], floor_factor * dmax);
    out.resid[q] = den > 0.0 ? cur[q] / den : 0.0;
    if (!(cur[q] <= thr[q])) out.converged = false;
  }
  return SMG_OK;
}

// ----------------------------------------------------------------------------
// DGF construction
// ----------------------------------------------------------------------------
namespace {

// device memory owned by the setup call
struct DevTmp {
  std::vector<void*> ptrs;
  ~DevTmp() {
    for (void* q : ptrs) (void)hipFree(q);
  }
  template <class T>
  T* upload(const std::vector<T>& v, hipStream_t st, hipError_t& err) {
    void* q = nullptr;
    err = hipMalloc(&q, std::max<size_t>(1, v.size() * sizeof(T)));
    if (err != hipSuccess) return nullptr;
    ptrs.push_back(q);
    if (!v.empty()) err = hipMemcpyAsync(q, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st);
    return static_cast<T*>(q);
  }
  void* alloc(size_t bytes, hipError_t& err) {
    void* q = nullptr;
    err = hipMalloc(&q, std::max<size_t>(1, bytes));
    if (err == hipSuccess) ptrs.push_back(q);
    return q;
  }
};

#define TMPCHK(ptr)                                                                                \
  do {                                                                                             \
    if (herr != hipSuccess || !(ptr))                                                              \
      return fail(SMG_EHIP, strprintf("device allocation/copy failed: %s", hipGetErrorString(herr))); \
  } while (0)

}  // namespace

static smg_status dgf_constants(const smg_plan& p, DevTmp& tmp, hipStream_t st, DgfConst& K) {
  const Spec& s = p.spec;
  std::vector<double> cosk(s.n_phi), s2(p.M);
  for (int k = 0; k < s.n_phi; ++k) cosk[k] = std::cos(2.0 * kPi * k / s.n_phi);
  for (int m = 0; m < p.M; ++m) s2[m] = mode_s2(s.n_phi, m);
  hipError_t herr;
  K.sph = s.sph() ? 1 : 0;
  K.n_phi = s.n_phi;
  K.n_g = p.n_g;
  K.G = s.G;
  K.cosk = tmp.upload(cosk, st, herr);
  TMPCHK(K.cosk);
  K.s2 = tmp.upload(s2, st, herr);
  TMPCHK(K.s2);
  return SMG_OK;
}

static smg_status dgf_aux(smg_plan& p, hipStream_t st) {
  const Spec& s = p.spec;
  const GhostSet& gh = p.gh;
  const int npad = p.opts.n_pad, h = npad - 1;
  DevTmp tmp;
  hipError_t herr;
  DgfConst K;
  STCHK(dgf_constants(p, tmp, st, K));
  // first radial cell whose inner face is positive
  long i_pos = 1;
  while (s.radial_face((double)(i_pos - 2)) > 0.0 && i_pos > -100000) --i_pos;
  std::vector<int> ilo(p.n_g), ihi(p.n_g), jlo(p.n_g), jhi(p.n_g), ealo(p.n_g), eblo(p.n_g), ebhi(p.n_g);
  long amin = 1L << 30, amax = -(1L << 30), bmin = 1L << 30, bmax = -(1L << 30);
  int max_n1 = 0, max_n2 = 0;
  for (int g = 0; g < p.n_g; ++g) {
    long lo = gh.gi[g] - h, hi = gh.gi[g] + h;
    int ea = EDGE_DIRICHLET;
    if (s.radial_face((double)(lo - 2)) <= 0.0) { lo = i_pos; ea = EDGE_NEUMANN; }
    long jl = gh.gj[g] - h, jh = gh.gj[g] + h;
    int el = EDGE_DIRICHLET, eh = EDGE_DIRICHLET;
    if (s.pole_lo() && jl <= 1) { jl = 1; el = EDGE_POLE; }
    if (s.pole_hi() && jh >= s.n_b) { jh = s.n_b; eh = EDGE_POLE; }
    if (s.sph()) {
      if (el == EDGE_DIRICHLET && s.b_face(jl - 2) < 0.0) return fail(SMG_EINVAL, "DGF box crosses theta = 0 away from a pole");
      if (eh == EDGE_DIRICHLET && s.b_face(jh + 1) > kPi) return fail(SMG_EINVAL, "DGF box crosses theta = pi away from a pole");
    }
    ilo[g] = (int)lo; ihi[g] = (int)hi; jlo[g] = (int)jl; jhi[g] = (int)jh;
    ealo[g] = ea; eblo[g] = el; ebhi[g] = eh;
    amin = std::min(amin, lo - 1); amax = std::max(amax, hi + 1);
    bmin = std::min(bmin, jl - 1); bmax = std::max(bmax, jh + 1);
    max_n1 = std::max(max_n1, (int)(hi - lo + 1));
    max_n2 = std::max(max_n2, (int)(jh - jl + 1));
  }
  // continued axes covering every box and its ring: local k = global - off
  Axis A = make_axis(s, 'a', amin, 1, (int)(amax - amin - 1));
  Axis B = make_axis(s, 'b', bmin, 1, (int)(bmax - bmin - 1));
  std::vector<double> nfA(A.n + 2, 0.0), faceA(A.n + 2, 0.0);
  for (int k = 0; k < A.n + 2; ++k) {
    double lo = A.face[k], hi = A.face[k + 1];
    faceA[k] = lo;
    nfA[k] = s.sph() ? 3.0 * lo * lo / (hi * hi * hi - lo * lo * lo) : 2.0 * lo / (hi * hi - lo * lo);
  }
  std::vector<double> RA(A.R.begin(), A.R.end()), PA(A.P.begin(), A.P.end()), PB(B.P.begin(), B.P.end());
  AuxBoxes X{};
  X.i_lo = tmp.upload(ilo, st, herr); TMPCHK(X.i_lo);
  X.i_hi = tmp.upload(ihi, st, herr); TMPCHK(X.i_hi);
  X.j_lo = tmp.upload(jlo, st, herr); TMPCHK(X.j_lo);
  X.j_hi = tmp.upload(jhi, st, herr); TMPCHK(X.j_hi);
  X.e_alo = tmp.upload(ealo, st, herr); TMPCHK(X.e_alo);
  X.e_blo = tmp.upload(eblo, st, herr); TMPCHK(X.e_blo);
  X.e_bhi = tmp.upload(ebhi, st, herr); TMPCHK(X.e_bhi);
  X.offA = (int)amin;
  X.offB = (int)bmin;
  X.centA = tmp.upload(A.cent, st, herr); TMPCHK(X.centA);
  X.faceA = tmp.upload(faceA, st, herr); TMPCHK(X.faceA);
  X.upA = tmp.upload(A.up, st, herr); TMPCHK(X.upA);
  X.dnA = tmp.upload(A.dn, st, herr); TMPCHK(X.dnA);
  X.RA = tmp.upload(RA, st, herr); TMPCHK(X.RA);
  X.PA = tmp.upload(PA, st, herr); TMPCHK(X.PA);
  X.nfA = tmp.upload(nfA, st, herr); TMPCHK(X.nfA);
  X.centB = tmp.upload(B.cent, st, herr); TMPCHK(X.centB);
  X.upB = tmp.upload(B.up, st, herr); TMPCHK(X.upB);
  X.dnB = tmp.upload(B.dn, st, herr); TMPCHK(X.dnB);
  X.PB = tmp.upload(PB, st, herr); TMPCHK(X.PB);
  X.gi = tmp.upload(gh.gi, st, herr); TMPCHK(X.gi);
  X.gj = tmp.upload(gh.gj, st, herr); TMPCHK(X.gj);
  X.ga = tmp.upload(gh.a, st, herr); TMPCHK(X.ga);
  X.gb = tmp.upload(gh.b, st, herr); TMPCHK(X.gb);
  X.gdv = tmp.upload(gh.dv3, st, herr); TMPCHK(X.gdv);
  // modes in chunks so a launch stays short
  std::vector<int> modes(p.M);
  for (int m = 0; m < p.M; ++m) modes[m] = m;
  int* d_modes = tmp.upload(modes, st, herr); TMPCHK(d_modes);
  double* d_res = static_cast<double*>(tmp.alloc(sizeof(double) * (size_t)p.M * p.n_g, herr)); TMPCHK(d_res);
  double* out = reinterpret_cast<double*>(p.ws + p.w_dgf);
  const int chunk = std::max(1, 8192 / std::max(1, p.n_g));
  const int max_sweeps = 20000;
  for (int m0 = 0; m0 < p.M; m0 += chunk) {
    const int nm = std::min(chunk, p.M - m0);
    HIPCHK(smgk::dgf_aux(K, X, d_modes + m0, nm, out + (size_t)m0 * p.n_g * p.n_g, p.opts.dgf_tol, max_sweeps,
                         d_res + (size_t)m0 * p.n_g, max_n1, max_n2, st));
  }
  std::vector<double> res((size_t)p.M * p.n_g);
  HIPCHK(hipMemcpyAsync(res.data(), d_res, sizeof(double) * res.size(), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  double worst = 0.0;
  for (double v : res) worst = std::max(worst, v);
  p.dgf_resid = worst;
  if (!(worst <= 1e3 * p.opts.dgf_tol))
    return fail(SMG_ENOCONV, strprintf("auxiliary-grid DGF solve stalled at relative residual %.3e", worst));
  return SMG_OK;
}

static smg_status dgf_extended(smg_plan& p, hipStream_t st) {
  const Spec& s = p.spec;
  const GhostSet& gh = p.gh;
  const int npad = p.opts.n_pad;
  DevTmp tmp;
  hipError_t herr;
  DgfConst K;
  STCHK(dgf_constants(p, tmp, st, K));
  const long a_lo = 1 - (s.n_a - npad);
  const int na = 2 * s.n_a;
  long b_lo;
  int nb;
  int edge[4] = {EDGE_NEUMANN, EDGE_DIRICHLET, EDGE_DIRICHLET, EDGE_DIRICHLET};
  if (s.pole_lo() && s.pole_hi()) {
    b_lo = 1; nb = s.n_b; edge[2] = EDGE_POLE; edge[3] = EDGE_POLE;
  } else {
    b_lo = 1 - s.n_b / 2; nb = 2 * s.n_b;
  }
  std::vector<int> modes(p.M);
  for (int m = 0; m < p.M; ++m) modes[m] = m;
  Hierarchy HE = build_hierarchy(s, a_lo, na, b_lo, nb, edge, modes, false);
  if (HE.lv.back().na * HE.lv.back().nb > kMaxCoarseCells) return fail(SMG_EINVAL, "extended DGF domain does not coarsen enough");
  // pack and upload its tables
  Blob B;
  std::vector<LevelOff> lo;
  for (const LevelTables& T : HE.lv) lo.push_back(pack_level(B, T));
  char* tb = static_cast<char*>(tmp.alloc(B.bytes.size(), herr)); TMPCHK(tb);
  HIPCHK(hipMemcpyAsync(tb, B.bytes.data(), B.bytes.size(), hipMemcpyHostToDevice, st));
  MGFields F;
  F.exact = true;
  for (size_t l = 0; l < HE.lv.size(); ++l) F.L.push_back(level_view(tb, lo[l], HE.lv[l], p.M));
  // box geometry for the right-hand sides
  const LevelTables& T0 = HE.lv[0];
  ExtBox E{};
  E.na = na; E.nb = nb;
  E.e_blo = edge[2] == EDGE_POLE ? 1 : 0;
  E.e_bhi = edge[3] == EDGE_POLE ? 1 : 0;
  E.centA = tmp.upload(T0.A.cent, st, herr); TMPCHK(E.centA);
  E.centB = tmp.upload(T0.B.cent, st, herr); TMPCHK(E.centB);
  E.RA = tmp.upload(T0.Rr, st, herr); TMPCHK(E.RA);
  {
    double l0 = T0.A.face[1], h0 = T0.A.face[2];
    E.face0 = l0;
    E.nfA = s.sph() ? 3.0 * l0 * l0 / (h0 * h0 * h0 - l0 * l0 * l0) : 2.0 * l0 / (h0 * h0 - l0 * l0);
  }
  E.upA_last = T0.A.up[na];
  E.dnB_first = T0.B.dn[1];
  E.upB_last = T0.B.up[nb];
  std::vector<int> cell(p.n_g);
  for (int g = 0; g < p.n_g; ++g) cell[g] = (int)((gh.gi[g] - a_lo) * nb + (gh.gj[g] - b_lo));
  E.cell = tmp.upload(cell, st, herr); TMPCHK(E.cell);
  E.ga = tmp.upload(gh.a, st, herr); TMPCHK(E.ga);
  E.gb = tmp.upload(gh.b, st, herr); TMPCHK(E.gb);
  E.gdv = tmp.upload(gh.dv3, st, herr); TMPCHK(E.gdv);
  // plane list: (mode, source pair), mode-major
  std::vector<int> pm, ps0, ps1;
  for (int m = 0; m < p.M; ++m)
    for (int g = 0; g < p.n_g; g += 2) {
      pm.push_back(m);
      ps0.push_back(g);
      ps1.push_back(g + 1 < p.n_g ? g + 1 : -1);
    }
  const int total = (int)pm.size();
  // chunk size from a memory budget for the level fields
  size_t per_plane = 0;
  for (const LevelTables& T : HE.lv) per_plane += 2 * sizeof(double2) * (size_t)T.na * T.nb;
  size_t budget = (size_t)4 << 30;
  int cap = (int)std::max<size_t>(1, std::min<size_t>(budget / per_plane, 4096));
  cap = std::min(cap, total);
  double2* u0 = static_cast<double2*>(tmp.alloc(sizeof(double2) * (size_t)cap * na * nb, herr)); TMPCHK(u0);
  double2* f0 = static_cast<double2*>(tmp.alloc(sizeof(double2) * (size_t)cap * na * nb, herr)); TMPCHK(f0);
  F.u.assign(HE.lv.size(), nullptr);
  F.f.assign(HE.lv.size(), nullptr);
  for (size_t l = 1; l < HE.lv.size(); ++l) {
    size_t pl = (size_t)HE.lv[l].na * HE.lv[l].nb;
    F.u[l] = static_cast<double2*>(tmp.alloc(sizeof(double2) * cap * pl, herr)); TMPCHK(F.u[l]);
    F.f[l] = static_cast<double2*>(tmp.alloc(sizeof(double2) * cap * pl, herr)); TMPCHK(F.f[l]);
  }
  plan_lds(F);
  int* d_slot = static_cast<int*>(tmp.alloc(sizeof(int) * cap, herr)); TMPCHK(d_slot);
  int* d_mode = static_cast<int*>(tmp.alloc(sizeof(int) * cap, herr)); TMPCHK(d_mode);
  int* d_pm = tmp.upload(pm, st, herr); TMPCHK(d_pm);
  int* d_s0 = tmp.upload(ps0, st, herr); TMPCHK(d_s0);
  int* d_s1 = tmp.upload(ps1, st, herr); TMPCHK(d_s1);
  double* d_partial = static_cast<double*>(tmp.alloc(sizeof(double) * cap * kNormBlocks, herr)); TMPCHK(d_partial);
  double* d_norm = static_cast<double*>(tmp.alloc(sizeof(double) * cap, herr)); TMPCHK(d_norm);
  int *h_slot = nullptr, *h_mode = nullptr;
  double* h_norm = nullptr;
  HIPCHK(hipHostMalloc((void**)&h_slot, sizeof(int) * cap));
  std::unique_ptr<int, void (*)(int*)> g1(h_slot, [](int* q) { (void)hipHostFree(q); });
  HIPCHK(hipHostMalloc((void**)&h_mode, sizeof(int) * cap));
  std::unique_ptr<int, void (*)(int*)> g2(h_mode, [](int* q) { (void)hipHostFree(q); });
  HIPCHK(hipHostMalloc((void**)&h_norm, sizeof(double) * cap));
  std::unique_ptr<double, void (*)(double*)> g3(h_norm, [](double* q) { (void)hipHostFree(q); });
  double* out = reinterpret_cast<double*>(p.ws + p.w_dgf);
  for (int q0 = 0; q0 < total; q0 += cap) {
    const int n = std::min(cap, total - q0);
    HIPCHK(smgk::dgf_ext_rhs(K, E, d_pm + q0, d_s0 + q0, d_s1 + q0, n, f0, st));
    SolveOut so;
    STCHK(mg_solve_planes(p, F, n, &pm[q0], u0, f0, p.opts.dgf_tol, 0.0, false, 100, d_slot, d_mode, h_slot, h_mode,
                          d_partial, d_norm, h_norm, st, so));
    for (double v : so.resid) p.dgf_resid = std::max(p.dgf_resid, v);
    if (!(p.dgf_resid <= 1e3 * p.opts.dgf_tol))
      return fail(SMG_ENOCONV, strprintf("extended-domain DGF solve stalled at relative residual %.3e", p.dgf_resid));
    HIPCHK(smgk::dgf_ext_extract(E, p.n_g, d_pm + q0, d_s0 + q0, d_s1 + q0, n, u0, out, st));
  }
  HIPCHK(hipStreamSynchronize(st));
  return SMG_OK;
}

// ----------------------------------------------------------------------------
// setup and solve
// ----------------------------------------------------------------------------
extern "C" smg_status smg_plan_setup(smg_plan* p, void* workspace, size_t bytes, void* stream) {
  if (!p) return fail(SMG_EINVAL, "NULL plan");
  if (!workspace || bytes < p->w_total) return fail(SMG_EWORKSPACE, strprintf("workspace of %zu bytes needed", p->w_total));
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return fail(SMG_EWORKSPACE, "workspace must be 256-byte aligned");
  hipStream_t st = static_cast<hipStream_t>(stream);
  p->ws = static_cast<char*>(workspace);
  p->ready = false;
  p->have_prev = false;
  if (!p->h_slot) HIPCHK(hipHostMalloc((void**)&p->h_slot, sizeof(int) * p->M));
  if (!p->h_mode) HIPCHK(hipHostMalloc((void**)&p->h_mode, sizeof(int) * p->M));
  if (!p->h_norm) HIPCHK(hipHostMalloc((void**)&p->h_norm, sizeof(double) * p->M));
  HIPCHK(hipMemcpyAsync(p->ws + p->w_blob, p->blob.bytes.data(), p->blob.bytes.size(), hipMemcpyHostToDevice, st));
  p->mg.L.clear();
  p->mg.exact = p->opts.line_solver == SMG_LINE_EXACT;
  p->mg.fp32 = p->opts.precision == SMG_MIXED;
  for (size_t l = 0; l < p->H.lv.size(); ++l) p->mg.L.push_back(level_view(p->ws + p->w_blob, p->loff[l], p->H.lv[l], p->M));
  p->mg.u.assign(p->H.lv.size(), nullptr);
  p->mg.f.assign(p->H.lv.size(), nullptr);
  for (size_t l = 1; l < p->H.lv.size(); ++l) {
    p->mg.u[l] = p->dptr(p->w_u[l]);
    p->mg.f[l] = p->dptr(p->w_fl[l]);
  }
  if (p->mg.fp32) {
    p->mg.u32.assign(p->H.lv.size(), nullptr);
    p->mg.f32.assign(p->H.lv.size(), nullptr);
    for (size_t l = 0; l < p->H.lv.size(); ++l) {
      p->mg.u32[l] = reinterpret_cast<float2*>(p->ws + p->w_u32[l]);
      p->mg.f32[l] = reinterpret_cast<float2*>(p->ws + p->w_f32[l]);
    }
  }
  plan_lds(p->mg);
  smg_status s = dgf_method_of(*p) == SMG_DGF_EXTENDED ? dgf_extended(*p, st) : dgf_aux(*p, st);
  if (s != SMG_OK) return s;
  HIPCHK(hipStreamSynchronize(st));
  p->ready = true;
  return SMG_OK;
}

static smg_status need_ready(const smg_plan* p) {
  if (!p) return fail(SMG_EINVAL, "NULL plan");
  if (!p->ready) return fail(SMG_ESTATE, "plan is not set up (call smg_plan_setup first)");
  return SMG_OK;
}

static smg_status solve_main(smg_plan* p, const double2* f, double2* u, double tol, bool warm, hipStream_t st,
                             SolveOut& so) {
  std::vector<int> modes(p->M);
  for (int m = 0; m < p->M; ++m) modes[m] = m;
  return mg_solve_planes(*p, p->mg, p->M, modes.data(), u, f, tol, kFloor, warm, p->opts.max_cycles,
                         reinterpret_cast<int*>(p->ws + p->w_slot), reinterpret_cast<int*>(p->ws + p->w_mode),
                         p->h_slot, p->h_mode, reinterpret_cast<double*>(p->ws + p->w_partial),
                         reinterpret_cast<double*>(p->ws + p->w_norm), p->h_norm, st, so);
}

static smg_status james_steps(smg_plan* p, const double2* psi, const double2* f, double2* sigma, double2* theta,
                              double2* f2, hipStream_t st) {
  const Spec& s = p->spec;
  const int plane = s.n_a * s.n_b;
  const char* base = p->ws + p->w_blob;
  const double M = p->M, ng = p->n_g;
  int ev = prof_mark(*p, st);
  HIPCHK(smgk::james_screen(reinterpret_cast<const int*>(base + p->o_adj), reinterpret_cast<const double*>(base + p->o_cout),
                            p->n_g, plane, p->M, psi, 1.0 / (4.0 * kPi * s.G), sigma, st));
  prof_close(*p, K_SCREEN, ev, M * ng * 32.0, st);
  ev = prof_mark(*p, st);
  HIPCHK(smgk::james_conv(reinterpret_cast<const double*>(p->ws + p->w_dgf), sigma, theta, p->n_g, p->M, st));
  prof_close(*p, K_CONV, ev, M * ng * ng * 8.0 + M * ng * 32.0, st);
  if (f2 != f) HIPCHK(hipMemcpyAsync(f2, f, sizeof(double2) * (size_t)p->M * plane, hipMemcpyDeviceToDevice, st));
  ev = prof_mark(*p, st);
  HIPCHK(smgk::james_apply(reinterpret_cast<const int*>(base + p->o_apc), reinterpret_cast<const int*>(base + p->o_apg0),
                           reinterpret_cast<const int*>(base + p->o_apg1), reinterpret_cast<const double*>(base + p->o_apc0),
                           reinterpret_cast<const double*>(base + p->o_apc1), (int)p->ap_cell.size(), plane, p->n_g,
                           p->M, theta, f2, f2, st));
  prof_close(*p, K_APPLY, ev, M * (double)p->ap_cell.size() * 48.0, st);
  return SMG_OK;
}

extern "C" smg_status smg_solve(smg_plan* p, const double* rho, double* phi, double tol, unsigned flags, void* stream,
                                smg_info* info) {
  STCHK(need_ready(p));
  if (!rho || !phi) return fail(SMG_EINVAL, "rho and phi must not be NULL");
  if (!(tol > 0.0)) return fail(SMG_EINVAL, "rel_tol must be > 0");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Spec& s = p->spec;
  const bool timings = (flags & SMG_TIMINGS) && info;
  hipEvent_t ev[6] = {};
  if (timings)
    for (auto& e : ev) HIPCHK(hipEventCreate(&e));
  struct EvGuard {
    hipEvent_t* e; bool on;
    ~EvGuard() { if (on) for (int k = 0; k < 6; ++k) (void)hipEventDestroy(e[k]); }
  } guard{ev, timings};
  const char* base = p->ws + p->w_blob;
  const double2* tw = reinterpret_cast<const double2*>(base + p->o_tw);
  double2* f = p->dptr(p->w_f);
  double2* psi = p->dptr(p->w_psi);
  double2* phim = p->dptr(p->w_phi);
  const bool warm = (flags & SMG_WARM_PREV) && p->have_prev;
  const int lines = s.n_a * s.n_b;
  if (timings) HIPCHK(hipEventRecord(ev[0], st));
  const double fft_bytes = (double)lines * (8.0 * s.n_phi + 16.0 * p->M);
  int pe = prof_mark(*p, st);
  HIPCHK(smgk::fft_r2c(rho, f, lines, s.n_phi, 4.0 * kPi * s.G / s.n_phi, tw, st));
  prof_close(*p, K_FFT_R2C, pe, fft_bytes, st);
  if (timings) HIPCHK(hipEventRecord(ev[1], st));
  SolveOut s1, s2;
  STCHK(solve_main(p, f, psi, tol, warm, st, s1));
  if (timings) HIPCHK(hipEventRecord(ev[2], st));
  STCHK(james_steps(p, psi, f, p->dptr(p->w_sigma), p->dptr(p->w_theta), f, st));
  if (timings) HIPCHK(hipEventRecord(ev[3], st));
  STCHK(solve_main(p, f, phim, tol, warm, st, s2));
  if (timings) HIPCHK(hipEventRecord(ev[4], st));
  pe = prof_mark(*p, st);
  HIPCHK(smgk::fft_c2r(phim, phi, lines, s.n_phi, tw, st));
  prof_close(*p, K_FFT_C2R, pe, fft_bytes, st);
  if (timings) HIPCHK(hipEventRecord(ev[5], st));
  p->have_prev = true;
  if (info) {
    HIPCHK(hipStreamSynchronize(st));
    info->n_modes = p->M;
    info->total_cycles = 0;
    for (int m = 0; m < p->M; ++m) {
      if (info->cycles1) info->cycles1[m] = s1.cycles[m];
      if (info->cycles2) info->cycles2[m] = s2.cycles[m];
      if (info->resid1) info->resid1[m] = s1.resid[m];
      if (info->resid2) info->resid2[m] = s2.resid[m];
      info->total_cycles += s1.cycles[m] + s2.cycles[m];
    }
    info->converged = (s1.converged && s2.converged) ? 1 : 0;
    if (timings) {
      float t[5];
      for (int k = 0; k < 5; ++k) HIPCHK(hipEventElapsedTime(&t[k], ev[k], ev[k + 1]));
      info->ms_fft = t[0]; info->ms_mg1 = t[1]; info->ms_james = t[2]; info->ms_mg2 = t[3]; info->ms_ifft = t[4];
    }
  }
  if (!(s1.converged && s2.converged)) return fail(SMG_ENOCONV, "a mode did not reach the tolerance within max_cycles");
  return SMG_OK;
}

// ----------------------------------------------------------------------------
// step-level entry points
// ----------------------------------------------------------------------------
extern "C" smg_status smg_fft_forward(smg_plan* p, const double* rho, double* modes, void* stream) {
  STCHK(need_ready(p));
  const Spec& s = p->spec;
  const double2* tw = reinterpret_cast<const double2*>(p->ws + p->w_blob + p->o_tw);
  HIPCHK(smgk::fft_r2c(rho, reinterpret_cast<double2*>(modes), s.n_a * s.n_b, s.n_phi, 4.0 * kPi * s.G / s.n_phi, tw,
                       static_cast<hipStream_t>(stream)));
  return SMG_OK;
}

extern "C" smg_status smg_fft_inverse(smg_plan* p, const double* modes, double* phi, void* stream) {
  STCHK(need_ready(p));
  const Spec& s = p->spec;
  const double2* tw = reinterpret_cast<const double2*>(p->ws + p->w_blob + p->o_tw);
  HIPCHK(smgk::fft_c2r(reinterpret_cast<const double2*>(modes), phi, s.n_a * s.n_b, s.n_phi, tw,
                       static_cast<hipStream_t>(stream)));
  return SMG_OK;
}

extern "C" smg_status smg_mg_solve(smg_plan* p, const double* f, double* u, double tol, void* stream, int* cycles,
                                   double* resid) {
  STCHK(need_ready(p));
  if (!(tol > 0.0)) return fail(SMG_EINVAL, "rel_tol must be > 0");
  SolveOut so;
  STCHK(solve_main(p, reinterpret_cast<const double2*>(f), reinterpret_cast<double2*>(u), tol, true,
                   static_cast<hipStream_t>(stream), so));
  for (int m = 0; m < p->M; ++m) {
    if (cycles) cycles[m] = so.cycles[m];
    if (resid) resid[m] = so.resid[m];
  }
  if (!so.converged) return fail(SMG_ENOCONV, "a mode did not reach the tolerance within max_cycles");
  return SMG_OK;
}

static Batch all_modes(smg_plan* p, hipStream_t st, hipError_t& e) {
  for (int m = 0; m < p->M; ++m) { p->h_slot[m] = m; p->h_mode[m] = m; }
  int* ds = reinterpret_cast<int*>(p->ws + p->w_slot);
  int* dm = reinterpret_cast<int*>(p->ws + p->w_mode);
  e = hipMemcpyAsync(ds, p->h_slot, sizeof(int) * p->M, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(dm, p->h_mode, sizeof(int) * p->M, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return Batch{p->M, ds, dm};
}

extern "C" smg_status smg_mg_vcycle(smg_plan* p, const double* f, double* u, void* stream) {
  STCHK(need_ready(p));
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e;
  Batch b = all_modes(p, st, e);
  HIPCHK(e);
  STCHK(vcycle(*p, p->mg, b, reinterpret_cast<double2*>(u), reinterpret_cast<const double2*>(f), st));
  return SMG_OK;
}

extern "C" smg_status smg_mg_smooth(smg_plan* p, const double* f, double* u, void* stream) {
  STCHK(need_ready(p));
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e;
  Batch b = all_modes(p, st, e);
  HIPCHK(e);
  HIPCHK(smgk::mg_smooth(p->mg.L[0], b, reinterpret_cast<double2*>(u), reinterpret_cast<const double2*>(f), p->opts.n_sor,
                         p->mg.exact, st));
  return SMG_OK;
}

extern "C" smg_status smg_mg_residual(smg_plan* p, const double* f, const double* u, double* r, void* stream) {
  STCHK(need_ready(p));
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e;
  Batch b = all_modes(p, st, e);
  HIPCHK(e);
  HIPCHK(smgk::mg_residual(p->mg.L[0], b, reinterpret_cast<const double2*>(u), reinterpret_cast<const double2*>(f),
                           reinterpret_cast<double2*>(r), st));
  return SMG_OK;
}

extern "C" smg_status smg_james(smg_plan* p, const double* psi, const double* f, double* sigma, double* theta, double* f2,
                                void* stream) {
  STCHK(need_ready(p));
  return james_steps(p, reinterpret_cast<const double2*>(psi), reinterpret_cast<const double2*>(f),
                     reinterpret_cast<double2*>(sigma), reinterpret_cast<double2*>(theta), reinterpret_cast<double2*>(f2),
                     static_cast<hipStream_t>(stream));
}

extern "C" smg_status smg_dgf_table(smg_plan* p, int m, double* host, void* stream) {
  STCHK(need_ready(p));
  if (m < 0 || m >= p->M || !host) return fail(SMG_EINVAL, "bad mode or NULL buffer");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t n = (size_t)p->n_g * p->n_g;
  HIPCHK(hipMemcpyAsync(host, p->ws + p->w_dgf + sizeof(double) * n * m, sizeof(double) * n, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return SMG_OK;
}

// ----------------------------------------------------------------------------
// per-launch timing entry points
// ----------------------------------------------------------------------------
extern "C" smg_status smg_profile_begin(smg_plan* p) {
  if (!p) return fail(SMG_EINVAL, "NULL plan");
  p->prof_on = true;
  p->prof_used = 0;
  p->prof_log.clear();
  return SMG_OK;
}

extern "C" smg_status smg_profile_end(smg_plan* p, smg_kernel_stat* stats, int max_stats, int* n_stats) {
  if (!p) return fail(SMG_EINVAL, "NULL plan");
  p->prof_on = false;
  HIPCHK(hipDeviceSynchronize());
  std::vector<int> launches(K_COUNT, 0);
  std::vector<double> ms(K_COUNT, 0.0), bytes(K_COUNT, 0.0);
  for (const auto& r : p->prof_log) {
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, p->prof_pool[r.ev0], p->prof_pool[r.ev1]));
    launches[r.cls] += 1;
    ms[r.cls] += t;
    bytes[r.cls] += r.bytes;
  }
  int n = 0;
  for (int c = 0; c < K_COUNT; ++c) {
    if (!launches[c]) continue;
    if (stats && n < max_stats) {
      stats[n].name = kKernelNames[c];
      stats[n].launches = launches[c];
      stats[n].total_ms = ms[c];
      stats[n].bytes = bytes[c];
    }
    ++n;
  }
  if (n_stats) *n_stats = n;
  p->prof_log.clear();
  p->prof_used = 0;
  return SMG_OK;
}
