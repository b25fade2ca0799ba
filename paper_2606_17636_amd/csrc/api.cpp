// C ABI of the smg library (include/smg.h): plan creation and validation,
// workspace layout, device setup (table upload, DGF construction), the
// batched multigrid driver and the seven-step solve of Sec. 5.1.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "dgf_dev.h"
#include "engine.h"
#include "netdef.h"
#include "netguess.h"
#include "smg_internal.h"

using namespace smg;

static thread_local std::string g_err;

static smg_status fail(smg_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

namespace smg {
void set_error(const std::string& msg) { g_err = msg; }
}  // namespace smg

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
      pb_w0, pb_w1, sep_v, sep_vi, sep_cp, sep_id;
  bool has_sep;
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
  o.has_sep = !T.sep_v.empty();
  o.sep_v = o.has_sep ? B.add(T.sep_v) : 0;
  o.sep_vi = o.has_sep ? B.add(T.sep_vi) : 0;
  o.sep_cp = o.has_sep ? B.add(T.sep_cp) : 0;
  o.sep_id = o.has_sep ? B.add(T.sep_id) : 0;
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
  L.sep_v = o.has_sep ? d(o.sep_v) : nullptr;
  L.sep_vi = o.has_sep ? d(o.sep_vi) : nullptr;
  L.sep_cp = o.has_sep ? d(o.sep_cp) : nullptr;
  L.sep_id = o.has_sep ? d(o.sep_id) : nullptr;
  return L;
}

}  // namespace

struct smg_plan;

namespace {
// Routes the engine's per-launch timing marks to the plan's event pool.
struct PlanProf : ProfSink {
  const smg_plan* p = nullptr;
  int mark(hipStream_t st) override;
  void close(int cls, int ev, double bytes, hipStream_t st) override;
  int launch_events(hipEvent_t* start, hipEvent_t* stop) override;
  void close_launch(int cls, int id, double bytes) override;
};

// A captured solve body (both multigrid solves and the boundary steps) for
// one per-cycle schedule.
struct GraphEnt {
  std::vector<int> key;
  hipGraphExec_t exec = nullptr;
  unsigned long long used = 0;
};
constexpr int kMaxGraphs = 64;
}  // namespace

// Plans whose multigrid solves share one engine (a plan alone, or a batch):
// per-mode cycle history, solve graphs and their capture stream.
struct Group {
  std::vector<smg_plan*> plans;
  Engine* eng = nullptr;
  int launch = SMG_LAUNCH_GRAPH;
  int max_cycles = 60;
  bool have_prev = false;
  // per-mode cycle counts of the last solve, per initial-guess kind and
  // target: the schedule of the next solve of that kind.  Kinds: 0 zero
  // guess; warm starts 1 + x + 5 g, with x the solutions the extrapolation
  // uses (0: none, 1: the previous one .. 4: cubic) and g = 1 with the
  // learned guess -- each start needs its own number of cycles
  static constexpr int kKinds = 11;
  std::vector<int> hist[kKinds][2];
  std::vector<int> hist_prev[kKinds][2];  // the counts of the solve of that kind before the last one
  int margin[kKinds] = {};                // extra cycles per mode: 1 after a solve of the kind ran short
  bool hist_ok[kKinds] = {};
  std::vector<GraphEnt> graphs;
  unsigned long long clock = 0;
  hipStream_t cap_stream = nullptr;  // private stream the solve graphs are captured on
  void drop_graphs() {
    for (GraphEnt& g : graphs)
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
    graphs.clear();
  }
  void reset() {
    have_prev = false;
    for (bool& b : hist_ok) b = false;
    for (auto& h : hist_prev)
      for (auto& v : h) v.clear();
    drop_graphs();
  }
  Group() = default;
  Group(const Group&) = delete;
  Group& operator=(const Group&) = delete;
  ~Group() {
    drop_graphs();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
  }
};

// The learned guess attached to a plan: network, caller-owned work buffer
// and the offsets of its parts.
struct PlanNet {
  smg_net* net = nullptr;
  int m_max = 0, n_img = 0, nblk = 1;
  char* work = nullptr;
  NetWork wl{};
  size_t o_fprev[2] = {0, 0}, o_uprev[2] = {0, 0}, o_uprev2[2] = {0, 0}, o_cand = 0, o_cs = 0, o_us = 0, o_u2 = 0,
         o_u2b = 0, o_sc = 0, o_part = 0, o_used = 0, o_jobs = 0, o_lv = 0, o_list = 0, o_rec = 0, o_rec0 = 0, o_scpart = 0, bytes = 0;
  std::vector<NormJob> hjobs;  // [target][smoothed candidate, smoothed previous solution]
  std::vector<LvJob> hlv;      // [target][the same two arrays]: one smoothing step
  bool prev_ok[2] = {false, false};
  // o_uprev[t] holds the solution one step back (set by the last guess
  // step of target t), so the next one can move it two steps back
  bool have_u[2] = {false, false};
  bool prev2_ok[2] = {false, false};   // the current guess step has u two steps back
  float* samples = nullptr;
  int capacity = 0;
};

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
  // face acceleration: inverse centroid distances and metric factors, ghost offsets
  size_t o_acc_da = 0, o_acc_db = 0, o_acc_ra = 0, o_acc_sb = 0;
  int acc_g_ahi = 0, acc_g_blo = -1, acc_g_bhi = -1;
  bool have_theta = false;  // w_theta holds the Theta of an enqueued solve
  // workspace layout (byte offsets)
  size_t w_blob = 0, w_dgf = 0, w_psi = 0, w_phi = 0, w_f = 0, w_f2 = 0, w_sigma = 0, w_theta = 0, w_gpot = 0, w_eng = 0,
         w_eng_bytes = 0, w_total = 0;
  std::vector<size_t> w_u, w_fl, w_u32, w_f32, w_u2;
  // bound workspace
  char* ws = nullptr;
  bool ready = false;
  double dgf_resid = 0.0;  // worst relative residual of the DGF solves
  std::vector<LevelDev> levels;
  Engine eng;               // targets: 0 = Psi (solve 1), 1 = Phi (solve 2)
  Group grp;                // this plan alone
  std::string tune_report;
  PlanNet pn;
  // extrapolated warm start (opts.warm_extrapolate = order): the solutions
  // before the last one per target (order of them), how many solutions of
  // the target the plan holds in a form a warm solve can use (0 .. order + 1:
  // w_psi/w_phi and w_xprev), and how many this solve extrapolates from (0:
  // no step, 1: only shift the history), decided on the host before the body
  size_t w_xprev[2][3] = {{0, 0, 0}, {0, 0, 0}};
  int xhave[2] = {0, 0};
  int xstep[2] = {0, 0};
  // the kept solutions live in a ring of slots: xorder[t][j] is the slot of
  // the j-th newest; a solve writes u_{t-1} into the oldest position's slot,
  // which then becomes the newest (no data moves); back to identity whenever
  // the history is empty again
  int xorder[2][3] = {{0, 1, 2}, {0, 1, 2}};
  // bumped whenever a buffer that captured solve graphs write to changes
  // (network attach, recording buffer); part of every group graph key, so a
  // batch holding this plan never replays a graph with the old pointers
  unsigned gen = 0;
  // per-launch event timing (smg_profile_begin / smg_profile_end)
  struct ProfRec { int cls, ev0, ev1; double bytes; };
  mutable bool prof_on = false;
  mutable std::vector<hipEvent_t> prof_pool;
  mutable size_t prof_used = 0;
  mutable std::vector<ProfRec> prof_log;
  PlanProf prof_sink;
  ~smg_plan() {
    for (hipEvent_t e : prof_pool) (void)hipEventDestroy(e);
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
  const bool nu_auto = o.nu_pre == SMG_NU_AUTO && o.nu_post == SMG_NU_AUTO;
  if (!nu_auto && (o.nu_pre < 0 || o.nu_post < 0 || o.nu_pre + o.nu_post < 1))
    return fail(SMG_EINVAL, "need nu_pre + nu_post >= 1 (or both SMG_NU_AUTO)");
  if (o.n_sor < 1 || o.max_cycles < 1) return fail(SMG_EINVAL, "need n_sor >= 1, max_cycles >= 1");
  if (o.n_pad < 2 || o.n_pad > 24) return fail(SMG_EINVAL, "n_pad must be in [2, 24]");
  if (o.dgf_method < SMG_DGF_AUTO || o.dgf_method > SMG_DGF_EXTENDED) return fail(SMG_EINVAL, "bad dgf_method");
  if (o.line_solver != SMG_LINE_SOR && o.line_solver != SMG_LINE_EXACT) return fail(SMG_EINVAL, "bad line_solver");
  if (o.coarse_cells != 0 && (o.coarse_cells < 16 || o.coarse_cells > 8192))
    return fail(SMG_EINVAL, "coarse_cells must be 0 or in [16, 8192]");
  if (o.coarse_solver != SMG_COARSE_EXACT && o.coarse_solver != SMG_COARSE_SOR)
    return fail(SMG_EINVAL, "coarse_solver must be SMG_COARSE_EXACT or SMG_COARSE_SOR");
  if (o.warm_extrapolate < 0 || o.warm_extrapolate > 3) return fail(SMG_EINVAL, "warm_extrapolate must be 0 to 3");
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
  p->H = build_hierarchy(s, 1, s.n_a, 1, s.n_b, edge, modes, true, o.coarse_cells,
                         o.coarse_solver == SMG_COARSE_EXACT);
  const LevelTables& Lc = p->H.lv.back();
  if (Lc.na * Lc.nb > kMaxCoarseCells && Lc.sep_v.empty())
    return fail(SMG_EINVAL, strprintf("the %dx%d coarsest level has no exact solver", Lc.na, Lc.nb));
  if (Lc.na * Lc.nb > std::max(kMaxCoarseCells, o.coarse_cells))
    return fail(SMG_EINVAL, strprintf("grid coarsens only to %dx%d (> %d cells): %s", Lc.na, Lc.nb,
                                      std::max(kMaxCoarseCells, o.coarse_cells), p->H.stop));
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
  // face acceleration tables (Eq. gradient): projected centroid distances
  // across the radial and theta/z faces (ghost centroids at the ends; a face
  // lying on a pole gets 0, i.e. g = 0), radial centroids and sin(theta)
  {
    const Axis A = make_axis(s, 'a', 0, 1, s.n_a), B = make_axis(s, 'b', 0, 1, s.n_b);
    std::vector<double> ida(s.n_a + 1), idb(s.n_b + 1), ira(s.n_a), isb(s.n_b);
    for (int f = 0; f <= s.n_a; ++f) ida[f] = 1.0 / (A.cent[f + 1] - A.cent[f]);
    for (int f = 0; f <= s.n_b; ++f) {
      const bool pole = (f == 0 && s.pole_lo()) || (f == s.n_b && s.pole_hi());
      idb[f] = pole ? 0.0 : 1.0 / (B.cent[f + 1] - B.cent[f]);
    }
    for (int i = 0; i < s.n_a; ++i) ira[i] = 1.0 / A.cent[i + 1];
    for (int j = 0; j < s.n_b; ++j) isb[j] = s.sph() ? 1.0 / std::sin(B.cent[j + 1]) : 1.0;
    p->o_acc_da = p->blob.add(ida);
    p->o_acc_db = p->blob.add(idb);
    p->o_acc_ra = p->blob.add(ira);
    p->o_acc_sb = p->blob.add(isb);
    // ghost order: inner radial (n_b), outer radial (n_b), lower b, upper b (n_a each, Dirichlet edges only)
    p->acc_g_ahi = s.n_b;
    p->acc_g_blo = s.pole_lo() ? -1 : 2 * s.n_b;
    p->acc_g_bhi = s.pole_hi() ? -1 : 2 * s.n_b + (s.pole_lo() ? 0 : s.n_a);
  }
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
  p->w_f2 = take(sizeof(double2) * M * plane);
  for (int k = 0; k < p->opts.warm_extrapolate; ++k)
    for (int t = 0; t < 2; ++t) p->w_xprev[t][k] = take(sizeof(double2) * M * plane);
  p->w_sigma = take(sizeof(double2) * (size_t)M * p->n_g);
  p->w_theta = take(sizeof(double2) * (size_t)M * p->n_g);
  p->w_gpot = take(sizeof(double) * (size_t)p->n_g * s.n_phi);
  p->w_eng_bytes = Engine::region_bytes(2, 1, (int)p->H.lv.size(), M);
  p->w_eng = take(p->w_eng_bytes);
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
  // second iterate array of the smoother per level (the cycle's type)
  p->w_u2.assign(p->H.lv.size(), 0);
  for (size_t l = 0; l < p->H.lv.size(); ++l) {
    size_t pl = (size_t)p->H.lv[l].na * p->H.lv[l].nb;
    p->w_u2[l] = take((o.precision == SMG_MIXED ? sizeof(float2) : sizeof(double2)) * M * pl);
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
  K_FFT_R2C, K_FFT_C2R, K_SMOOTH_RADIAL0, K_SMOOTH_POLAR0, K_SMOOTH_RADIAL_C, K_SMOOTH_POLAR_C, K_RESTRICT,
  K_PROLONG, K_COARSE, K_NORM, K_SCREEN, K_CONV, K_APPLY, K_ACCUM, K_COUNT
};
static const char* kKernelNames[K_COUNT] = {
  "fft_r2c", "fft_c2r", "smooth_radial_lines_l0", "smooth_polar_lines_l0", "smooth_radial_lines_coarser",
  "smooth_polar_lines_coarser",
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

int PlanProf::mark(hipStream_t st) { return prof_mark(*p, st); }

// two pool events, not recorded here: the launch records them
static int prof_take(const smg_plan& p) {
  if (!p.prof_on) return -1;
  while (p.prof_pool.size() < p.prof_used + 2) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return -1;
    p.prof_pool.push_back(e);
  }
  p.prof_used += 2;
  return (int)p.prof_used - 2;
}

int PlanProf::launch_events(hipEvent_t* start, hipEvent_t* stop) {
  const int id = prof_take(*p);
  if (id < 0) return -1;
  *start = p->prof_pool[id];
  *stop = p->prof_pool[id + 1];
  return id;
}

void PlanProf::close(int cls, int ev, double bytes, hipStream_t st) {
  static const int map[] = {K_SMOOTH_RADIAL0, K_SMOOTH_POLAR0, K_SMOOTH_RADIAL_C, K_SMOOTH_POLAR_C, K_RESTRICT,
                            K_PROLONG,        K_COARSE,        K_NORM,            K_ACCUM,           K_NORM};
  prof_close(*p, map[cls], ev, bytes, st);
}

void PlanProf::close_launch(int cls, int id, double bytes) {
  static const int map[] = {K_SMOOTH_RADIAL0, K_SMOOTH_POLAR0, K_SMOOTH_RADIAL_C, K_SMOOTH_POLAR_C, K_RESTRICT,
                            K_PROLONG,        K_COARSE,        K_NORM,            K_ACCUM,           K_NORM};
  if (id >= 0) p->prof_log.push_back({map[cls], id, id + 1, bytes});
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
  std::vector<LevelDev> LV;
  for (size_t l = 0; l < HE.lv.size(); ++l) LV.push_back(level_view(tb, lo[l], HE.lv[l], p.M));
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
  int cap = (int)std::max<size_t>(1, std::min<size_t>(budget / per_plane, (size_t)Engine::kMaxPlanes));
  cap = std::min(cap, total);
  // the list is padded to whole chunks; padding planes get a zero source and
  // drop out at once (zero defect)
  const int chunks = (total + cap - 1) / cap;
  pm.resize((size_t)chunks * cap, 0);
  ps0.resize((size_t)chunks * cap, -1);
  ps1.resize((size_t)chunks * cap, -1);
  const size_t box = (size_t)na * nb;
  double2* u0 = static_cast<double2*>(tmp.alloc(sizeof(double2) * (size_t)cap * box, herr)); TMPCHK(u0);
  double2* f0 = static_cast<double2*>(tmp.alloc(sizeof(double2) * (size_t)cap * box, herr)); TMPCHK(f0);
  int* d_pm = tmp.upload(pm, st, herr); TMPCHK(d_pm);
  int* d_s0 = tmp.upload(ps0, st, herr); TMPCHK(d_s0);
  int* d_s1 = tmp.upload(ps1, st, herr); TMPCHK(d_s1);
  int* d_mode = static_cast<int*>(tmp.alloc(sizeof(int) * cap, herr)); TMPCHK(d_mode);
  MGProblem pr;
  pr.L = LV;
  pr.u.assign(HE.lv.size(), nullptr);
  pr.f.assign(HE.lv.size(), nullptr);
  pr.u2.assign(HE.lv.size(), nullptr);
  for (size_t l = 0; l < HE.lv.size(); ++l) {
    size_t pl = (size_t)HE.lv[l].na * HE.lv[l].nb;
    pr.u2[l] = tmp.alloc(sizeof(double2) * cap * pl, herr); TMPCHK(pr.u2[l]);
    if (l == 0) continue;
    pr.u[l] = tmp.alloc(sizeof(double2) * cap * pl, herr); TMPCHK(pr.u[l]);
    pr.f[l] = tmp.alloc(sizeof(double2) * cap * pl, herr); TMPCHK(pr.f[l]);
  }
  pr.u0 = {u0};
  pr.f0 = {f0};
  pr.mode = d_mode;
  pr.n = cap;
  MGParams prm;
  prm.nu_pre = p.opts.nu_pre;
  prm.nu_post = p.opts.nu_post;
  prm.n_sor = p.opts.n_sor;
  prm.exact = true;
  prm.fp32 = false;
  prm.coarse_rtol = kCoarseRtol;
  prm.coarse_sweeps = kCoarseSweeps;
  const size_t eb = Engine::region_bytes(1, 1, (int)HE.lv.size(), cap);
  char* er = static_cast<char*>(tmp.alloc(eb, herr)); TMPCHK(er);
  Engine eng;
  std::string emsg;
  smg_status es = eng.init({pr}, 1, prm, er, eb, st, &emsg);
  if (es != SMG_OK) return fail(es, "extended DGF engine: " + emsg);
  double* out = reinterpret_cast<double*>(p.ws + p.w_dgf);
  std::vector<int> cyc;
  std::vector<double> cur, thr, d0;
  for (int q0 = 0; q0 < total; q0 += cap) {
    const int n = std::min(cap, total - q0);
    HIPCHK(hipMemcpyAsync(d_mode, d_pm + q0, sizeof(int) * cap, hipMemcpyDeviceToDevice, st));
    HIPCHK(smgk::fill_zero(f0, (size_t)cap * box, st));
    HIPCHK(smgk::dgf_ext_rhs(K, E, d_pm + q0, d_s0 + q0, d_s1 + q0, n, f0, st));
    STCHK(eng.start(0, p.opts.dgf_tol, 0.0, false, 100, st));
    STCHK(eng.finish_dynamic(0, st, nullptr));
    STCHK(eng.read_state(0, st, cyc, cur, thr, d0));
    for (int k = 0; k < n; ++k)
      if (d0[k] > 0.0) p.dgf_resid = std::max(p.dgf_resid, cur[k] / d0[k]);
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
// The plan's multigrid as the engine sees it: targets 0 (Psi, right-hand
// side f) and 1 (Phi^m, right-hand side f2).
static MGProblem plan_problem(smg_plan* p) {
  const bool fp32 = p->opts.precision == SMG_MIXED;
  const int L = (int)p->H.lv.size();
  MGProblem pr;
  pr.L = p->levels;
  pr.u.assign(L, nullptr);
  pr.f.assign(L, nullptr);
  for (int l = 0; l < L; ++l) {
    if (fp32) {
      pr.u[l] = p->ws + p->w_u32[l];
      pr.f[l] = p->ws + p->w_f32[l];
    } else if (l > 0) {
      pr.u[l] = p->dptr(p->w_u[l]);
      pr.f[l] = p->dptr(p->w_fl[l]);
    }
  }
  pr.u2.assign(L, nullptr);
  for (int l = 0; l < L; ++l) pr.u2[l] = p->ws + p->w_u2[l];
  pr.u0 = {p->dptr(p->w_psi), p->dptr(p->w_phi)};
  pr.f0 = {p->dptr(p->w_f), p->dptr(p->w_f2)};
  if (fp32) {
    pr.r32 = reinterpret_cast<float2*>(p->ws + p->w_f32[0]);
    pr.e32 = reinterpret_cast<float2*>(p->ws + p->w_u32[0]);
  }
  pr.n = p->M;
  return pr;
}

static MGParams plan_params(const smg_plan* p) {
  MGParams prm;
  prm.nu_pre = p->opts.nu_pre;
  prm.nu_post = p->opts.nu_post;
  prm.n_sor = p->opts.n_sor;
  prm.exact = p->opts.line_solver == SMG_LINE_EXACT;
  prm.fp32 = p->opts.precision == SMG_MIXED;
  prm.coarse_rtol = kCoarseRtol;
  prm.coarse_sweeps = kCoarseSweeps;
  return prm;
}

extern "C" smg_status smg_plan_setup(smg_plan* p, void* workspace, size_t bytes, void* stream) {
  if (!p) return fail(SMG_EINVAL, "NULL plan");
  if (!workspace || bytes < p->w_total) return fail(SMG_EWORKSPACE, strprintf("workspace of %zu bytes needed", p->w_total));
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return fail(SMG_EWORKSPACE, "workspace must be 256-byte aligned");
  hipStream_t st = static_cast<hipStream_t>(stream);
  p->ws = static_cast<char*>(workspace);
  p->ready = false;
  p->grp.reset();
  p->xhave[0] = p->xhave[1] = 0;
  HIPCHK(hipMemcpyAsync(p->ws + p->w_blob, p->blob.bytes.data(), p->blob.bytes.size(), hipMemcpyHostToDevice, st));
  p->levels.clear();
  for (size_t l = 0; l < p->H.lv.size(); ++l)
    p->levels.push_back(level_view(p->ws + p->w_blob, p->loff[l], p->H.lv[l], p->M));
  MGProblem pr = plan_problem(p);
  MGParams prm = plan_params(p);
  std::string emsg;
  smg_status es = p->eng.init({pr}, 2, prm, p->ws + p->w_eng, p->w_eng_bytes, st, &emsg);
  if (es != SMG_OK) return fail(es, "multigrid engine: " + emsg);
  p->prof_sink.p = p;
  p->eng.set_prof(&p->prof_sink);
  p->grp.plans = {p};
  p->grp.eng = &p->eng;
  p->grp.launch = p->opts.launch;
  p->grp.max_cycles = p->opts.max_cycles;
  smg_status s = dgf_method_of(*p) == SMG_DGF_EXTENDED ? dgf_extended(*p, st) : dgf_aux(*p, st);
  if (s != SMG_OK) return s;
  if (p->opts.autotune) {
    // the tuning cycles run on a zero right-hand side (launch times do not
    // depend on the values)
    HIPCHK(smgk::fill_zero(p->dptr(p->w_f), (size_t)p->M * p->spec.n_a * p->spec.n_b, st));
    STCHK(p->eng.start(0, 1e-8, kFloor, false, 1, st));
    const bool was = p->prof_on;
    p->prof_on = false;
    es = p->eng.autotune(0, st, &p->tune_report);
    p->prof_on = was;
    if (es != SMG_OK) return fail(es, "autotune: " + p->tune_report);
  }
  HIPCHK(hipStreamSynchronize(st));
  p->ready = true;
  return SMG_OK;
}

static smg_status need_ready(const smg_plan* p) {
  if (!p) return fail(SMG_EINVAL, "NULL plan");
  if (!p->ready) return fail(SMG_ESTATE, "plan is not set up (call smg_plan_setup first)");
  return SMG_OK;
}

// f2_holds_f: f2 already holds f (the forward FFT wrote both), so only the
// boundary cells are completed.
static smg_status james_steps(smg_plan* p, const double2* psi, const double2* f, double2* sigma, double2* theta,
                              double2* f2, hipStream_t st, bool f2_holds_f = false) {
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
  if (f2 != f && !f2_holds_f) HIPCHK(smgk::copy_planes(f2, f, (size_t)p->M * plane, st));
  ev = prof_mark(*p, st);
  HIPCHK(smgk::james_apply(reinterpret_cast<const int*>(base + p->o_apc), reinterpret_cast<const int*>(base + p->o_apg0),
                           reinterpret_cast<const int*>(base + p->o_apg1), reinterpret_cast<const double*>(base + p->o_apc0),
                           reinterpret_cast<const double*>(base + p->o_apc1), (int)p->ap_cell.size(), plane, p->n_g,
                           p->M, theta, f2, f2, st));
  prof_close(*p, K_APPLY, ev, M * (double)p->ap_cell.size() * 48.0, st);
  return SMG_OK;
}

// Per-cycle plane counts of a solve from the per-mode cycle counts of the
// previous one: cycle k runs on the modes that needed more than k cycles.
// Every mode is given as many cycles as it needed in the more demanding of
// the last two solves of the kind (a sequence whose counts alternate, a
// time series of warm starts, is covered; a repeated solve is scheduled
// exactly), plus `margin` after a solve that ran short.  A mode that
// converges early drops out of the device list (its blocks return at once);
// one cycle too few sends the whole solve back to the host loop.
static std::vector<int> schedule_of(const std::vector<int>& cyc, const std::vector<int>& prev, int margin) {
  std::vector<int> need(cyc);
  if (prev.size() == cyc.size())
    for (size_t k = 0; k < need.size(); ++k) need[k] = std::max(need[k], prev[k]);
  for (int& c : need) c += margin;
  int mx = 0;
  for (int c : need) mx = std::max(mx, c);
  std::vector<int> caps(mx, 0);
  for (int c : need)
    for (int k = 0; k < c; ++k) caps[k] += 1;
  return caps;
}

// f2_holds_f: every plan's solve-2 right-hand side still holds the
// transformed density (written by fft_forward_all, not completed since).
static smg_status james_all(Group& g, hipStream_t st, bool f2_holds_f) {
  for (smg_plan* p : g.plans) {
    STCHK(james_steps(p, p->dptr(p->w_psi), p->dptr(p->w_f), p->dptr(p->w_sigma), p->dptr(p->w_theta),
                      p->dptr(p->w_f2), st, f2_holds_f));
    p->have_theta = true;
  }
  return SMG_OK;
}

// ---- the learned guess inside a solve --------------------------------------
static const double2* target_f(const smg_plan* p, int t) { return p->dptr(t == 0 ? p->w_f : p->w_f2); }
static double2* target_u(const smg_plan* p, int t) { return p->dptr(t == 0 ? p->w_psi : p->w_phi); }

// Before solve t of a warm start: the network inputs of modes 0..m_max;
// with `guess`, the candidate (the linear extrapolation of the last two
// solutions plus s_o net(x)) replaces the previous step's solution in every
// mode where, after one smoothing step of each, its defect norm is the
// smaller one.
static smg_status net_before(smg_plan* p, int t, bool warm, bool guess, hipStream_t st) {
  PlanNet& pn = p->pn;
  if (!pn.net || !warm || !pn.prev_ok[t]) return SMG_OK;
  // the inputs serve the network's guess or a recorded sample, nothing else
  if (!guess && !pn.samples) return SMG_OK;
  const int plane = p->spec.n_a * p->spec.n_b;
  const size_t np = (size_t)(pn.m_max + 1) * plane;
  double2* uprev = reinterpret_cast<double2*>(pn.work + pn.o_uprev[t]);
  double2* uprev2 = reinterpret_cast<double2*>(pn.work + pn.o_uprev2[t]);
  double* sc = reinterpret_cast<double*>(pn.work + pn.o_sc);
  const double2* fprev = reinterpret_cast<const double2*>(pn.work + pn.o_fprev[t]);
  // the host decided before the body (group_solve) whether uprev still holds
  // the solution of the step before the previous one
  if (pn.prev2_ok[t]) HIPCHK(smgk::copy_planes(uprev2, uprev, np, st));
  HIPCHK(smgk::copy_planes(uprev, target_u(p, t), np, st));
  HIPCHK(smgg::scales(target_f(p, t), fprev, uprev, pn.prev2_ok[t] ? uprev2 : nullptr, plane, pn.n_img,
                      reinterpret_cast<double*>(pn.work + pn.o_scpart), sc, st));
  HIPCHK(smgg::assemble(target_f(p, t), fprev, uprev, pn.prev2_ok[t] ? uprev2 : nullptr, sc, p->spec.n_a, p->spec.n_b,
                        pn.n_img, reinterpret_cast<float*>(pn.work + pn.wl.x32), st));
  if (!guess) return SMG_OK;
  STCHK(pn.net->def.forward(pn.work, pn.wl, st, false));
  // the candidate (also into the copy the judge smooths) and the baseline
  // it is judged against (the linear extrapolation, or the previous solution
  // before two exist), the latter straight into the judge's second buffer
  HIPCHK(smgg::candidate(uprev, pn.prev2_ok[t] ? uprev2 : nullptr, reinterpret_cast<const float*>(pn.work + pn.wl.y), sc,
                         plane, pn.m_max, reinterpret_cast<double2*>(pn.work + pn.o_cand),
                         reinterpret_cast<double2*>(pn.work + pn.o_us), st,
                         reinterpret_cast<double2*>(pn.work + pn.o_cs)));
  return SMG_OK;
}

// Second phase of the learned guess of solve t: the judge.  The candidate
// and the other start each get one smoothing step and the one with the
// smaller defect norm is kept.  The other start is the baseline of
// net_before, or, where the plan's extrapolated warm start has already
// written u (base_in_u), u itself: the candidate then has to beat the
// plan's own start.  (The smoothing removes the rough part of an error,
// which the multigrid removes in its first sweep anyway; what is left
// decides the cycles.)
static smg_status net_judge(smg_plan* p, int t, bool warm, bool guess, bool base_in_u, hipStream_t st) {
  PlanNet& pn = p->pn;
  if (!pn.net || !warm || !pn.prev_ok[t] || !guess) return SMG_OK;
  const int plane = p->spec.n_a * p->spec.n_b;
  const size_t np = (size_t)(pn.m_max + 1) * plane;
  const double2* uprev = reinterpret_cast<const double2*>(pn.work + pn.o_uprev[t]);
  const double2* uprev2 = reinterpret_cast<const double2*>(pn.work + pn.o_uprev2[t]);
  const double* sc = reinterpret_cast<const double*>(pn.work + pn.o_sc);
  const double2* cand = reinterpret_cast<const double2*>(pn.work + pn.o_cand);
  if (base_in_u) HIPCHK(smgk::copy_planes(reinterpret_cast<double2*>(pn.work + pn.o_us), target_u(p, t), np, st));
  // both starts as the two problems of one launch per step: list position
  // q (m_max + 1) + m is start q's mode m, so the norm partials of the
  // candidate come first, then those of the other start
  BatchRef b{2 * (pn.m_max + 1), nullptr, reinterpret_cast<const int*>(pn.work + pn.o_list)};
  const LvJob* dl = reinterpret_cast<const LvJob*>(pn.work + pn.o_lv) + 2 * t;
  const bool exact = p->opts.line_solver == SMG_LINE_EXACT;
  for (int dir = 0; dir < 2; ++dir)
    HIPCHK(smgk::mg_smooth_dir(dl, &pn.hlv[2 * t], 2, b, p->opts.n_sor, exact, dir, false, st));
  const NormJob* dj = reinterpret_cast<const NormJob*>(pn.work + pn.o_jobs) + 2 * t;
  double* pc = reinterpret_cast<double*>(pn.work + pn.o_part);
  double* pu = pc + (size_t)(pn.m_max + 1) * pn.nblk;
  HIPCHK(smgk::mg_norm_partial(dj, &pn.hjobs[2 * t], 2, b, true, pc, pn.nblk, st));
  HIPCHK(smgg::select(pc, pu, pn.nblk, cand, base_in_u ? nullptr : uprev, pn.prev2_ok[t] ? uprev2 : nullptr, sc,
                      target_u(p, t), plane, pn.m_max, reinterpret_cast<int*>(pn.work + pn.o_used) + t * (pn.m_max + 1),
                      st));
  return SMG_OK;
}

// After solve t: a training sample per image when recording (from the
// third step of a sequence on), and this step's right-hand side kept for
// the next step's inputs.
static smg_status net_after(smg_plan* p, int t, bool warm, hipStream_t st) {
  PlanNet& pn = p->pn;
  if (!pn.net) return SMG_OK;
  const int plane = p->spec.n_a * p->spec.n_b;
  // samples only where the candidate extrapolates (two solutions back
  // exist): the network learns one kind of correction
  if (warm && pn.prev_ok[t] && pn.prev2_ok[t] && pn.samples)
    HIPCHK(smgg::record(reinterpret_cast<const float*>(pn.work + pn.wl.x32), target_u(p, t),
                        reinterpret_cast<const double2*>(pn.work + pn.o_uprev[t]),
                        pn.prev2_ok[t] ? reinterpret_cast<const double2*>(pn.work + pn.o_uprev2[t]) : nullptr,
                        reinterpret_cast<const double*>(pn.work + pn.o_sc), plane, pn.n_img,
                        reinterpret_cast<int*>(pn.work + pn.o_rec), pn.capacity, pn.samples, st));
  // solve 1's inputs are built only while samples are recorded, so its
  // right-hand side is kept only then
  if (t == 0 && !pn.samples) {
    pn.prev_ok[0] = false;
    return SMG_OK;
  }
  HIPCHK(smgk::copy_planes(reinterpret_cast<double2*>(pn.work + pn.o_fprev[t]), target_f(p, t),
                           (size_t)(pn.m_max + 1) * plane, st));
  pn.prev_ok[t] = true;
  return SMG_OK;
}

// The body of a solve between the two FFTs: solve 1 into Psi, the James
// steps, solve 2 into Phi^m, for every plan of the group (with the learned
// guess of plans that carry a network).  With schedules, every cycle is
// enqueued up front (no host synchronisation); otherwise each solve reads
// its list length after every cycle.  ev (optional) records 3 component
// boundaries.
// Extrapolated warm start of target t (decided on the host: p->xstep[t]
// solutions to extrapolate from): every mode starts from the polynomial
// extrapolation of its last solutions (order 1: 2 u_{t-1} - u_{t-2};
// 2: 3 u_{t-1} - 3 u_{t-2} + u_{t-3}; 3: 4 u_{t-1} - 6 u_{t-2} + 4 u_{t-3} -
// u_{t-4}), and the kept history advances (the kernel writes u_{t-1} into
// the oldest position's slot; group_solve rotates the slot order after the
// solve).  Runs between the two phases of the
// learned guess: after net_before has read u_{t-1}, before the judge, which
// then weighs the network's candidate against this start.
static smg_status warm_extrapolate(smg_plan* p, int t, bool warm, hipStream_t st) {
  if (!warm || p->xstep[t] == 0) return SMG_OK;
  const size_t plane = (size_t)p->spec.n_a * p->spec.n_b, n = (size_t)p->M * plane;
  const int kept = p->opts.warm_extrapolate;
  double2* hist[3] = {nullptr, nullptr, nullptr};
  for (int j = 0; j < kept; ++j) hist[j] = p->dptr(p->w_xprev[t][p->xorder[t][j]]);
  HIPCHK(smgg::extrapolate(target_u(p, t), hist, kept, n, 0, p->xstep[t], st));
  return SMG_OK;
}

static smg_status group_body(Group& g, double tol, bool warm, unsigned flags, const std::vector<int>* sched0,
                             const std::vector<int>* sched1, hipStream_t st, hipEvent_t* ev) {
  Engine& e = *g.eng;
  const bool guess = (flags & SMG_NET_GUESS) != 0;
  for (smg_plan* p : g.plans)  // samples of a solve the host has to finish are withdrawn (group_solve)
    if (p->pn.net && p->pn.samples)
      HIPCHK(hipMemcpyAsync(p->pn.work + p->pn.o_rec0, p->pn.work + p->pn.o_rec, sizeof(int), hipMemcpyDeviceToDevice, st));
  // the network guesses the potential's solve (solve 2) only; solve 1 (Psi,
  // zero ghosts) keeps the network's bookkeeping and starts like the other modes
  for (smg_plan* p : g.plans) STCHK(net_before(p, 0, warm, false, st));
  for (smg_plan* p : g.plans) STCHK(warm_extrapolate(p, 0, warm, st));
  STCHK(e.start(0, tol, kFloor, warm, g.max_cycles, st));
  if (sched0) {
    for (int cap : *sched0) STCHK(e.cycle(0, cap, st));
  } else {
    STCHK(e.finish_dynamic(0, st, nullptr));
  }
  for (smg_plan* p : g.plans) STCHK(net_after(p, 0, warm, st));
  if (ev) HIPCHK(hipEventRecord(ev[0], st));
  STCHK(james_all(g, st, true));
  if (ev) HIPCHK(hipEventRecord(ev[1], st));
  for (smg_plan* p : g.plans) STCHK(net_before(p, 1, warm, guess, st));
  for (smg_plan* p : g.plans) STCHK(warm_extrapolate(p, 1, warm, st));
  for (smg_plan* p : g.plans) STCHK(net_judge(p, 1, warm, guess, p->xstep[1] >= 2, st));
  STCHK(e.start(1, tol, kFloor, warm, g.max_cycles, st));
  if (sched1) {
    for (int cap : *sched1) STCHK(e.cycle(1, cap, st));
  } else {
    STCHK(e.finish_dynamic(1, st, nullptr));
  }
  for (smg_plan* p : g.plans) STCHK(net_after(p, 1, warm, st));
  if (ev) HIPCHK(hipEventRecord(ev[2], st));
  return SMG_OK;
}

// Captured graph of group_body for the two schedules (cached).
static smg_status group_graph(Group& g, double tol, bool warm, unsigned flags, const std::vector<int>& s0,
                              const std::vector<int>& s1, hipGraphExec_t* out) {
  std::vector<int> key;
  key.push_back(warm ? 1 : 0);
  key.push_back((int)(flags & SMG_NET_GUESS));
  for (const smg_plan* p : g.plans) {  // the learned-guess steps the body holds
    key.push_back(p->pn.net ? 1 + 2 * p->pn.prev_ok[0] + 4 * p->pn.prev_ok[1] + 8 * (p->pn.samples != nullptr) +
                                  16 * p->pn.prev2_ok[0] + 32 * p->pn.prev2_ok[1]
                            : 0);
    key.push_back((int)p->gen);
    key.push_back(p->xstep[0] + 4 * p->xstep[1] + 16 * p->xorder[0][0] + 64 * p->xorder[1][0]);
  }
  long long tb;
  std::memcpy(&tb, &tol, sizeof(tb));
  key.push_back((int)(tb & 0xffffffff));
  key.push_back((int)(tb >> 32));
  key.push_back((int)s0.size());
  key.insert(key.end(), s0.begin(), s0.end());
  key.insert(key.end(), s1.begin(), s1.end());
  for (GraphEnt& ge : g.graphs)
    if (ge.key == key) {
      ge.used = ++g.clock;
      *out = ge.exec;
      return SMG_OK;
    }
  // captured on the group's own stream (the caller's may be the null
  // stream, which cannot capture) and launched on the caller's
  if (!g.cap_stream) HIPCHK(hipStreamCreateWithFlags(&g.cap_stream, hipStreamNonBlocking));
  hipGraph_t graph = nullptr;
  HIPCHK(hipStreamBeginCapture(g.cap_stream, hipStreamCaptureModeThreadLocal));
  smg_status sb = group_body(g, tol, warm, flags, &s0, &s1, g.cap_stream, nullptr);
  hipError_t ce = hipStreamEndCapture(g.cap_stream, &graph);
  if (sb != SMG_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return sb;
  }
  HIPCHK(ce);
  hipGraphExec_t exec = nullptr;
  hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  HIPCHK(ie);
  if ((int)g.graphs.size() >= kMaxGraphs) {
    auto lru = std::min_element(g.graphs.begin(), g.graphs.end(),
                                [](const GraphEnt& a, const GraphEnt& b) { return a.used < b.used; });
    (void)hipGraphExecDestroy(lru->exec);
    g.graphs.erase(lru);
  }
  g.graphs.push_back(GraphEnt{key, exec, ++g.clock});
  *out = exec;
  return SMG_OK;
}

static smg_status fft_forward_all(Group& g, const double* const* rho, hipStream_t st) {
  for (size_t q = 0; q < g.plans.size(); ++q) {
    smg_plan* p = g.plans[q];
    const Spec& s = p->spec;
    const int lines = s.n_a * s.n_b;
    const double2* tw = reinterpret_cast<const double2*>(p->ws + p->w_blob + p->o_tw);
    int pe = prof_mark(*p, st);
    // the solve-2 right-hand side starts as the same modes (the James steps
    // then complete its boundary cells in place)
    HIPCHK(smgk::fft_r2c(rho[q], p->dptr(p->w_f), lines, s.n_phi, 4.0 * kPi * s.G / s.n_phi, tw, st, p->dptr(p->w_f2)));
    prof_close(*p, K_FFT_R2C, pe, (double)lines * (8.0 * s.n_phi + 32.0 * p->M), st);
  }
  return SMG_OK;
}

static smg_status fft_inverse_all(Group& g, double* const* phi, hipStream_t st) {
  for (size_t q = 0; q < g.plans.size(); ++q) {
    smg_plan* p = g.plans[q];
    const Spec& s = p->spec;
    const int lines = s.n_a * s.n_b;
    const double2* tw = reinterpret_cast<const double2*>(p->ws + p->w_blob + p->o_tw);
    int pe = prof_mark(*p, st);
    HIPCHK(smgk::fft_c2r(p->dptr(p->w_phi), phi[q], lines, s.n_phi, tw, st));
    prof_close(*p, K_FFT_C2R, pe, (double)lines * (8.0 * s.n_phi + 16.0 * p->M), st);
  }
  return SMG_OK;
}

// The seven steps for every plan of the group.  infos: one per plan or NULL.
static smg_status group_solve(Group& g, const double* const* rho, double* const* phi, double tol, unsigned flags,
                              hipStream_t st, smg_info* infos, bool profiling) {
  const int P = (int)g.plans.size();
  for (int q = 0; q < P; ++q)
    if (!rho[q] || !phi[q]) return fail(SMG_EINVAL, "rho and phi must not be NULL");
  if (!(tol > 0.0)) return fail(SMG_EINVAL, "rel_tol must be > 0");
  const bool timings = (flags & SMG_TIMINGS) && infos;
  hipEvent_t ev[6] = {};
  if (timings)
    for (auto& e : ev) HIPCHK(hipEventCreate(&e));
  struct EvGuard {
    hipEvent_t* e; bool on;
    ~EvGuard() { if (on) for (int k = 0; k < 6; ++k) (void)hipEventDestroy(e[k]); }
  } guard{ev, timings};
  const bool warm = (flags & SMG_WARM_PREV) && g.have_prev;
  const bool extrap = (flags & SMG_WARM_EXTRAP) != 0;
  int xs = 0;  // solutions the extrapolated starts use (the most over the plans)
  for (smg_plan* p : g.plans) {
    if (extrap && !p->opts.warm_extrapolate)
      return fail(SMG_EINVAL, "SMG_WARM_EXTRAP needs a plan created with opts.warm_extrapolate");
    for (int t = 0; t < 2; ++t) {
      p->xstep[t] = extrap && warm ? std::min(p->xhave[t], p->opts.warm_extrapolate + 1) : 0;
      xs = std::max(xs, p->xstep[t]);
      if (p->xhave[t] <= 1)  // nothing kept yet: start the ring over (the same graphs for every sequence)
        for (int j = 0; j < 3; ++j) p->xorder[t][j] = j;
    }
  }
  const int wk = warm ? 1 + xs + ((flags & SMG_NET_GUESS) ? 5 : 0) : 0;
  // learned-guess bookkeeping, decided on the host (a replayed graph runs
  // none of the body's host code): a guess step of target t (the network's
  // inputs, and its candidate where it guesses) runs when the solve is warm,
  // the previous right-hand side is kept and the network guesses this
  // target (the potential's solve) or samples are recorded; it sees the
  // solution two steps back when the previous solve ran one as well
  std::vector<std::array<bool, 2>> guess_step(P, std::array<bool, 2>{false, false});
  for (int q = 0; q < P; ++q) {
    PlanNet& pn = g.plans[q]->pn;
    for (int t = 0; t < 2; ++t) {
      const bool inputs = pn.samples != nullptr || (t == 1 && (flags & SMG_NET_GUESS));
      guess_step[q][t] = pn.net && warm && pn.prev_ok[t] && inputs;
      pn.prev2_ok[t] = guess_step[q][t] && pn.have_u[t];
    }
  }
  // scheduled launches (one host synchronisation per solve) once a previous
  // solve of the same kind gave the per-mode cycle counts; per-cycle host
  // reads for the first solve and with SMG_LAUNCH_DYNAMIC.  Component timings
  // and per-launch profiling enqueue the scheduled launches from the host
  // instead of replaying the graph (the same launches, with events between)
  const bool sched = g.launch == SMG_LAUNCH_GRAPH && g.hist_ok[wk];
  const bool graph = sched && !timings && !profiling;
  if (timings) HIPCHK(hipEventRecord(ev[0], st));
  STCHK(fft_forward_all(g, rho, st));
  if (timings) HIPCHK(hipEventRecord(ev[1], st));
  std::vector<int> s0, s1;
  if (sched) {
    s0 = schedule_of(g.hist[wk][0], g.hist_prev[wk][0], g.margin[wk]);
    s1 = schedule_of(g.hist[wk][1], g.hist_prev[wk][1], g.margin[wk]);
  }
  if (graph) {
    hipGraphExec_t exec = nullptr;
    STCHK(group_graph(g, tol, warm, flags, s0, s1, &exec));
    HIPCHK(hipGraphLaunch(exec, st));
  } else {
    STCHK(group_body(g, tol, warm, flags, sched ? &s0 : nullptr, sched ? &s1 : nullptr, st, timings ? ev + 2 : nullptr));
  }
  STCHK(fft_inverse_all(g, phi, st));
  if (timings) HIPCHK(hipEventRecord(ev[5], st));
  g.have_prev = true;
  for (smg_plan* p : g.plans)
    for (int t = 0; t < 2; ++t) {
      p->xhave[t] = p->xstep[t] > 0 ? std::min(p->xstep[t] + 1, p->opts.warm_extrapolate + 1) : 1;
      const int kept = p->opts.warm_extrapolate;
      if (p->xstep[t] > 0 && kept > 1) {  // the oldest position's slot now holds the newest solution
        const int s0 = p->xorder[t][kept - 1];
        for (int j = kept - 1; j > 0; --j) p->xorder[t][j] = p->xorder[t][j - 1];
        p->xorder[t][0] = s0;
      }
    }
  for (int q = 0; q < P; ++q)
    for (int t = 0; t < 2; ++t) g.plans[q]->pn.have_u[t] = guess_step[q][t];
  // per-mode state of both solves (one synchronisation); modes that needed
  // more cycles than the schedule gave them are finished here and the
  // inverse transforms are repeated
  Engine& e = *g.eng;
  Engine::State es;
  STCHK(e.read_all(st, &es));
  if (sched) g.margin[wk] = (es.count[0] > 0 || es.count[1] > 0) ? 1 : 0;
  if (es.count[0] > 0 || es.count[1] > 0) {
    // the training samples recorded in the body came from unfinished solves
    for (smg_plan* p : g.plans)
      if (p->pn.net && p->pn.samples)
        HIPCHK(hipMemcpyAsync(p->pn.work + p->pn.o_rec, p->pn.work + p->pn.o_rec0, sizeof(int), hipMemcpyDeviceToDevice,
                              st));
    if (es.count[0] > 0) {
      STCHK(e.finish_dynamic(0, st, nullptr));
      STCHK(james_all(g, st, false));
      // Phi^m holds the result for the old boundary data: a good guess
      STCHK(e.start(1, tol, kFloor, true, g.max_cycles, st));
    }
    STCHK(e.finish_dynamic(1, st, nullptr));
    STCHK(fft_inverse_all(g, phi, st));
    STCHK(e.read_all(st, &es));
  }
  bool converged = true;
  for (int t = 0; t < 2; ++t)
    for (int k = 0; k < e.n_planes(); ++k)
      if (!(es.cur[t][k] <= es.thr[t][k])) converged = false;
  if (converged && g.launch == SMG_LAUNCH_GRAPH) {
    // a mode that took more cycles than scheduled keeps its new count
    for (int t = 0; t < 2; ++t) {
      g.hist_prev[wk][t] = g.hist[wk][t];
      g.hist[wk][t] = es.cyc[t];
    }
    g.hist_ok[wk] = true;
  }
  if (infos) {
    float t[5] = {0, 0, 0, 0, 0};
    if (timings)
      for (int k = 0; k < 5; ++k) HIPCHK(hipEventElapsedTime(&t[k], ev[k], ev[k + 1]));
    for (int q = 0; q < P; ++q) {
      smg_info* info = infos + q;
      const int M = g.plans[q]->M, b0 = e.base(q);
      info->n_modes = M;
      info->total_cycles = 0;
      bool ok = true;
      for (int m = 0; m < M; ++m) {
        const int k = b0 + m;
        const double den0 = es.thr[0][k] / tol, den1 = es.thr[1][k] / tol;
        if (info->cycles1) info->cycles1[m] = es.cyc[0][k];
        if (info->cycles2) info->cycles2[m] = es.cyc[1][k];
        if (info->resid1) info->resid1[m] = den0 > 0.0 ? es.cur[0][k] / den0 : 0.0;
        if (info->resid2) info->resid2[m] = den1 > 0.0 ? es.cur[1][k] / den1 : 0.0;
        info->total_cycles += es.cyc[0][k] + es.cyc[1][k];
        if (!(es.cur[0][k] <= es.thr[0][k]) || !(es.cur[1][k] <= es.thr[1][k])) ok = false;
      }
      info->converged = ok ? 1 : 0;
      if (timings) {
        info->ms_fft = t[0]; info->ms_mg1 = t[1]; info->ms_james = t[2]; info->ms_mg2 = t[3]; info->ms_ifft = t[4];
      }
    }
  }
  if (!converged) return fail(SMG_ENOCONV, "a mode did not reach the tolerance within max_cycles");
  return SMG_OK;
}

extern "C" smg_status smg_solve(smg_plan* p, const double* rho, double* phi, double tol, unsigned flags, void* stream,
                                smg_info* info) {
  STCHK(need_ready(p));
  return group_solve(p->grp, &rho, &phi, tol, flags, static_cast<hipStream_t>(stream), info, p->prof_on);
}

// ----------------------------------------------------------------------------
// the learned guess: attach a network, record training samples
// ----------------------------------------------------------------------------
static smg_status net_layout(const smg_plan* p, const smg_net* net, int m_max, PlanNet& pn) {
  if (!net) return fail(SMG_EINVAL, "NULL net");
  const int q = 1 << (net->def.levels - 1);
  if (m_max < 0 || m_max > 8 || m_max >= p->M) return fail(SMG_EINVAL, "m_max must be in [0, min(8, n_phi/2)]");
  if (p->spec.n_a % q || p->spec.n_b % q)
    return fail(SMG_EINVAL, strprintf("the network needs n_a and n_b divisible by %d", q));
  pn.m_max = m_max;
  pn.n_img = 2 * m_max + 1;
  pn.wl = net->def.work_layout(pn.n_img, p->spec.n_a, p->spec.n_b);
  const size_t plane = (size_t)p->spec.n_a * p->spec.n_b, np = (size_t)(m_max + 1) * plane;
  size_t off = align_up(pn.wl.bytes);
  auto take = [&](size_t b) { size_t o = off; off = align_up(off + b); return o; };
  pn.o_fprev[0] = take(sizeof(double2) * np);
  pn.o_fprev[1] = take(sizeof(double2) * np);
  for (int t = 0; t < 2; ++t) {
    pn.o_uprev[t] = take(sizeof(double2) * np);
    pn.o_uprev2[t] = take(sizeof(double2) * np);
  }
  pn.o_cand = take(sizeof(double2) * np);
  pn.o_cs = take(sizeof(double2) * np);
  pn.o_us = take(sizeof(double2) * np);
  // the smoother's second arrays of the two judged starts (smoothed in one launch)
  pn.o_u2 = take(sizeof(double2) * np);
  pn.o_u2b = take(sizeof(double2) * np);
  pn.o_sc = take(sizeof(double) * 4 * pn.n_img);
  pn.o_scpart = take(sizeof(double) * smgg::scales_partial_doubles(pn.n_img));
  NormJob hj{};
  hj.L = p->levels.empty() ? LevelDev{} : p->levels[0];
  pn.nblk = smgk::norm_blocks(&hj, 1);
  pn.o_part = take(sizeof(double) * 2 * (m_max + 1) * pn.nblk);
  pn.o_used = take(sizeof(int) * 2 * (m_max + 1));
  pn.o_jobs = take(sizeof(NormJob) * 4);
  pn.o_lv = take(sizeof(LvJob) * 4);
  pn.o_list = take(sizeof(int) * 2 * (m_max + 1));  // both starts' planes
  pn.o_rec = take(sizeof(int));
  pn.o_rec0 = take(sizeof(int));   // the count when the current solve started
  pn.bytes = off;
  return SMG_OK;
}

extern "C" size_t smg_plan_net_work_bytes(const smg_plan* p, const smg_net* net, int m_max) {
  if (!p || !net) return 0;
  PlanNet pn;
  if (net_layout(p, net, m_max, pn) != SMG_OK) return 0;
  return pn.bytes;
}

extern "C" smg_status smg_plan_attach_net(smg_plan* p, smg_net* net, int m_max, void* work, size_t bytes, void* stream) {
  STCHK(need_ready(p));
  p->grp.drop_graphs();
  ++p->gen;
  if (!net) {
    p->pn = PlanNet{};
    return SMG_OK;
  }
  if (!net->state) return fail(SMG_ESTATE, "net state not bound");
  PlanNet pn;
  STCHK(net_layout(p, net, m_max, pn));
  if (!work || bytes < pn.bytes) return fail(SMG_EWORKSPACE, strprintf("net work buffer of %zu bytes needed", pn.bytes));
  if (reinterpret_cast<uintptr_t>(work) % kAlign) return fail(SMG_EWORKSPACE, "net work buffer must be 256-byte aligned");
  hipStream_t st = static_cast<hipStream_t>(stream);
  pn.net = net;
  pn.work = static_cast<char*>(work);
  const bool exact = p->opts.line_solver == SMG_LINE_EXACT;
  for (int t = 0; t < 2; ++t) {
    for (size_t arr : {pn.o_cs, pn.o_us}) {
      const size_t u2 = arr == pn.o_cs ? pn.o_u2 : pn.o_u2b;
      NormJob c{};
      c.L = p->levels[0];
      c.u = reinterpret_cast<double2*>(pn.work + arr);
      c.f = target_f(p, t);
      pn.hjobs.push_back(c);
      LvJob J{};
      J.L = p->levels[0];
      J.C = p->levels[0];
      J.u = c.u;
      J.u2 = pn.work + u2;
      J.f = const_cast<double2*>(c.f);
      J.active = 1;
      for (int dir = 0; dir < 2; ++dir) {
        smgk::SmoothShape sh{};
        if (!smgk::smooth_shape(p->levels[0], dir, exact, false, 512, m_max + 1, &sh))
          return fail(SMG_EINVAL, "smoothing step of the guess does not fit in LDS");
        J.tile[dir] = sh.tile;
        J.ntile[dir] = sh.ntile;
        J.scratch[dir] = sh.scratch;
      }
      pn.hlv.push_back(J);
    }
  }
  // the judge's launches cover both starts: problem 0 the candidate, 1 the
  // other start, modes 0..m_max of each
  std::vector<int> list(2 * (m_max + 1));
  for (int m = 0; m <= m_max; ++m) {
    list[m] = ent_make(0, m);
    list[m_max + 1 + m] = ent_make(1, m);
  }
  std::vector<int> zeros(2 * (m_max + 1) + 1, 0);
  HIPCHK(hipMemcpyAsync(pn.work + pn.o_jobs, pn.hjobs.data(), sizeof(NormJob) * 4, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(pn.work + pn.o_lv, pn.hlv.data(), sizeof(LvJob) * 4, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(pn.work + pn.o_list, list.data(), sizeof(int) * list.size(), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(pn.work + pn.o_used, zeros.data(), sizeof(int) * 2 * (m_max + 1), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(pn.work + pn.o_rec, zeros.data(), sizeof(int), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  p->pn = pn;
  return SMG_OK;
}

extern "C" smg_status smg_plan_record(smg_plan* p, float* samples, int capacity, void* stream) {
  STCHK(need_ready(p));
  if (!p->pn.net) return fail(SMG_ESTATE, "no network attached (smg_plan_attach_net)");
  p->grp.drop_graphs();
  ++p->gen;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int zero = 0;
  HIPCHK(hipMemcpyAsync(p->pn.work + p->pn.o_rec, &zero, sizeof(int), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  p->pn.samples = capacity > 0 ? samples : nullptr;
  p->pn.capacity = capacity > 0 && samples ? capacity : 0;
  return SMG_OK;
}

extern "C" int smg_plan_recorded(const smg_plan* p, void* stream) {
  if (!p || !p->pn.net) return 0;
  int n = 0;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (hipMemcpyAsync(&n, p->pn.work + p->pn.o_rec, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess) return -1;
  if (hipStreamSynchronize(st) != hipSuccess) return -1;
  return n;
}

extern "C" smg_status smg_plan_net_used(const smg_plan* p, int* used, void* stream) {
  if (!p || !p->pn.net || !used) return fail(SMG_EINVAL, "no network attached or NULL buffer");
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIPCHK(hipMemcpyAsync(used, p->pn.work + p->pn.o_used, sizeof(int) * 2 * (p->pn.m_max + 1), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return SMG_OK;
}

extern "C" smg_status smg_net_guess_step(smg_plan* p, int t, const double* f, const double* fprev, const double* uprev,
                                         const double* uprev2, double* guess, float* x_out, float* y_out, int* used_host,
                                         void* stream) {
  STCHK(need_ready(p));
  PlanNet& pn = p->pn;
  if (!pn.net) return fail(SMG_ESTATE, "no network attached (smg_plan_attach_net)");
  if (t != 0 && t != 1) return fail(SMG_EINVAL, "t must be 0 (Psi) or 1 (Phi)");
  if (!f || !fprev || !uprev || !guess) return fail(SMG_EINVAL, "f, fprev, uprev and guess must not be NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t np = (size_t)(pn.m_max + 1) * p->spec.n_a * p->spec.n_b;
  HIPCHK(smgk::copy_planes(const_cast<double2*>(target_f(p, t)), reinterpret_cast<const double2*>(f), np, st));
  HIPCHK(smgk::copy_planes(reinterpret_cast<double2*>(pn.work + pn.o_fprev[t]), reinterpret_cast<const double2*>(fprev), np,
                           st));
  HIPCHK(smgk::copy_planes(target_u(p, t), reinterpret_cast<const double2*>(uprev), np, st));
  // net_before moves o_uprev (the solution one step back) two steps back
  if (uprev2)
    HIPCHK(smgk::copy_planes(reinterpret_cast<double2*>(pn.work + pn.o_uprev[t]), reinterpret_cast<const double2*>(uprev2),
                             np, st));
  const bool keep = pn.prev_ok[t];
  pn.prev_ok[t] = true;
  pn.prev2_ok[t] = uprev2 != nullptr;
  smg_status sb = net_before(p, t, true, true, st);
  if (sb == SMG_OK) sb = net_judge(p, t, true, true, false, st);
  pn.prev_ok[t] = keep;
  pn.prev2_ok[t] = false;
  pn.have_u[0] = pn.have_u[1] = false;
  // the plan's solve state now holds these planes: the next solve starts cold
  p->grp.have_prev = false;
  p->xhave[0] = p->xhave[1] = 0;
  STCHK(sb);
  HIPCHK(smgk::copy_planes(reinterpret_cast<double2*>(guess), target_u(p, t), np, st));
  const size_t img = (size_t)pn.n_img * p->spec.n_a * p->spec.n_b;
  if (x_out) HIPCHK(hipMemcpyAsync(x_out, pn.work + pn.wl.x32, sizeof(float) * img * 8, hipMemcpyDeviceToDevice, st));
  if (y_out) HIPCHK(hipMemcpyAsync(y_out, pn.work + pn.wl.y, sizeof(float) * img, hipMemcpyDeviceToDevice, st));
  if (used_host)
    HIPCHK(hipMemcpyAsync(used_host, pn.work + pn.o_used + sizeof(int) * t * (pn.m_max + 1), sizeof(int) * (pn.m_max + 1),
                          hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return SMG_OK;
}

// ----------------------------------------------------------------------------
// batches of plans: one engine over every plan's planes
// ----------------------------------------------------------------------------
struct smg_batch {
  std::vector<smg_plan*> plans;
  Engine eng;
  Group grp;
  int n_total = 0, max_levels = 0;
  size_t w_total = 0;
  bool ready = false;
  std::string tune_report;
};

extern "C" smg_status smg_batch_create(smg_plan* const* plans, int n_plans, smg_batch** out) {
  if (!plans || !out) return fail(SMG_EINVAL, "plans and out must not be NULL");
  *out = nullptr;
  if (n_plans < 1 || n_plans > 256) return fail(SMG_EINVAL, "a batch holds 1 to 256 plans");
  std::unique_ptr<smg_batch> b(new (std::nothrow) smg_batch());
  if (!b) return fail(SMG_EINVAL, "out of host memory");
  const smg_opts& o0 = plans[0] ? plans[0]->opts : smg_opts{};
  for (int q = 0; q < n_plans; ++q) {
    smg_plan* p = plans[q];
    if (!p) return fail(SMG_EINVAL, "NULL plan in batch");
    for (int r = 0; r < q; ++r)
      if (plans[r] == p) return fail(SMG_EINVAL, "a plan appears twice in the batch");
    const smg_opts& o = p->opts;
    if (o.precision != o0.precision || o.line_solver != o0.line_solver || o.nu_pre != o0.nu_pre ||
        o.nu_post != o0.nu_post || o.n_sor != o0.n_sor)
      return fail(SMG_EINVAL, "plans of a batch must share precision, line solver, nu_pre, nu_post and n_sor");
    b->plans.push_back(p);
    b->n_total += p->M;
    b->max_levels = std::max(b->max_levels, (int)p->H.lv.size());
  }
  if (b->n_total > Engine::kMaxPlanes) return fail(SMG_EINVAL, strprintf("a batch holds at most %d mode planes", Engine::kMaxPlanes));
  b->w_total = Engine::region_bytes(2, n_plans, b->max_levels, b->n_total);
  *out = b.release();
  return SMG_OK;
}

extern "C" size_t smg_batch_workspace_bytes(const smg_batch* b) { return b ? b->w_total : 0; }

extern "C" smg_status smg_batch_setup(smg_batch* b, void* workspace, size_t bytes, void* stream) {
  if (!b) return fail(SMG_EINVAL, "NULL batch");
  if (!workspace || bytes < b->w_total) return fail(SMG_EWORKSPACE, strprintf("workspace of %zu bytes needed", b->w_total));
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return fail(SMG_EWORKSPACE, "workspace must be 256-byte aligned");
  hipStream_t st = static_cast<hipStream_t>(stream);
  b->ready = false;
  b->grp.reset();
  std::vector<MGProblem> probs;
  for (smg_plan* p : b->plans) {
    if (!p->ready) return fail(SMG_ESTATE, "every plan of a batch must be set up first");
    probs.push_back(plan_problem(p));
  }
  std::string emsg;
  smg_status es = b->eng.init(probs, 2, plan_params(b->plans[0]), static_cast<char*>(workspace), bytes, st, &emsg);
  if (es != SMG_OK) return fail(es, "batch engine: " + emsg);
  b->grp.plans = b->plans;
  b->grp.eng = &b->eng;
  b->grp.launch = b->plans[0]->opts.launch;
  b->grp.max_cycles = 0;
  for (smg_plan* p : b->plans) b->grp.max_cycles = std::max(b->grp.max_cycles, p->opts.max_cycles);
  if (b->plans[0]->opts.autotune) {
    for (smg_plan* p : b->plans)
      HIPCHK(smgk::fill_zero(p->dptr(p->w_f), (size_t)p->M * p->spec.n_a * p->spec.n_b, st));
    STCHK(b->eng.start(0, 1e-8, kFloor, false, 1, st));
    es = b->eng.autotune(0, st, &b->tune_report);
    if (es != SMG_OK) return fail(es, "autotune: " + b->tune_report);
  }
  HIPCHK(hipStreamSynchronize(st));
  b->ready = true;
  return SMG_OK;
}

extern "C" smg_status smg_batch_solve(smg_batch* b, const double* const* rho, double* const* phi, double tol,
                                      unsigned flags, void* stream, smg_info* infos) {
  if (!b) return fail(SMG_EINVAL, "NULL batch");
  if (!b->ready) return fail(SMG_ESTATE, "batch is not set up (call smg_batch_setup first)");
  if (!rho || !phi) return fail(SMG_EINVAL, "rho and phi must not be NULL");
  for (smg_plan* p : b->plans)
    if (!p->ready) return fail(SMG_ESTATE, "a plan of the batch is no longer set up");
  return group_solve(b->grp, rho, phi, tol, flags, static_cast<hipStream_t>(stream), infos, false);
}

extern "C" const char* smg_batch_tune_report(const smg_batch* b) { return b ? b->tune_report.c_str() : ""; }

extern "C" smg_status smg_batch_destroy(smg_batch* b) {
  delete b;
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

// The step entry points work on copies in the plan's solve-1 arrays (the
// next smg_solve does not warm-start from them).
static smg_status stage_in(smg_plan* p, const double* f, const double* u, hipStream_t st) {
  const size_t n = (size_t)p->M * p->spec.n_a * p->spec.n_b;
  if (f) HIPCHK(smgk::copy_planes(p->dptr(p->w_f), reinterpret_cast<const double2*>(f), n, st));
  if (u) HIPCHK(smgk::copy_planes(p->dptr(p->w_psi), reinterpret_cast<const double2*>(u), n, st));
  p->grp.have_prev = false;
  p->xhave[0] = p->xhave[1] = 0;
  return SMG_OK;
}

static smg_status stage_out(smg_plan* p, double* u, hipStream_t st) {
  const size_t n = (size_t)p->M * p->spec.n_a * p->spec.n_b;
  HIPCHK(smgk::copy_planes(reinterpret_cast<double2*>(u), p->dptr(p->w_psi), n, st));
  return SMG_OK;
}

extern "C" smg_status smg_mg_solve(smg_plan* p, const double* f, double* u, double tol, void* stream, int* cycles,
                                   double* resid) {
  STCHK(need_ready(p));
  if (!f || !u) return fail(SMG_EINVAL, "f and u must not be NULL");
  if (!(tol > 0.0)) return fail(SMG_EINVAL, "rel_tol must be > 0");
  hipStream_t st = static_cast<hipStream_t>(stream);
  STCHK(stage_in(p, f, u, st));
  STCHK(p->eng.start(0, tol, kFloor, true, p->opts.max_cycles, st));
  STCHK(p->eng.finish_dynamic(0, st, nullptr));
  std::vector<int> cyc;
  std::vector<double> cur, thr, d0;
  STCHK(p->eng.read_state(0, st, cyc, cur, thr, d0));
  STCHK(stage_out(p, u, st));
  bool ok = true;
  for (int m = 0; m < p->M; ++m) {
    const double den = thr[m] / tol;
    if (cycles) cycles[m] = cyc[m];
    if (resid) resid[m] = den > 0.0 ? cur[m] / den : 0.0;
    if (!(cur[m] <= thr[m])) ok = false;
  }
  HIPCHK(hipStreamSynchronize(st));
  if (!ok) return fail(SMG_ENOCONV, "a mode did not reach the tolerance within max_cycles");
  return SMG_OK;
}

static smg_status need_fp64(const smg_plan* p) {
  if (p->opts.precision != SMG_FP64) return fail(SMG_EINVAL, "this step entry point needs an FP64 plan");
  return SMG_OK;
}

extern "C" smg_status smg_mg_vcycle(smg_plan* p, const double* f, double* u, void* stream) {
  STCHK(need_ready(p));
  STCHK(need_fp64(p));
  hipStream_t st = static_cast<hipStream_t>(stream);
  STCHK(stage_in(p, f, u, st));
  STCHK(p->eng.vcycle_all(0, p->M, (int)p->eng.configs().size() - 1, st));
  STCHK(stage_out(p, u, st));
  HIPCHK(hipStreamSynchronize(st));
  return SMG_OK;
}

extern "C" smg_status smg_mg_smooth(smg_plan* p, const double* f, double* u, void* stream) {
  STCHK(need_ready(p));
  STCHK(need_fp64(p));
  hipStream_t st = static_cast<hipStream_t>(stream);
  STCHK(stage_in(p, f, u, st));
  STCHK(p->eng.smooth_all(0, st));
  STCHK(stage_out(p, u, st));
  HIPCHK(hipStreamSynchronize(st));
  return SMG_OK;
}

extern "C" smg_status smg_mg_residual(smg_plan* p, const double* f, const double* u, double* r, void* stream) {
  STCHK(need_ready(p));
  STCHK(need_fp64(p));
  hipStream_t st = static_cast<hipStream_t>(stream);
  STCHK(stage_in(p, f, u, st));
  STCHK(p->eng.residual_all(0, reinterpret_cast<double2*>(r), st));
  HIPCHK(hipStreamSynchronize(st));
  return SMG_OK;
}

extern "C" smg_status smg_james(smg_plan* p, const double* psi, const double* f, double* sigma, double* theta, double* f2,
                                void* stream) {
  STCHK(need_ready(p));
  return james_steps(p, reinterpret_cast<const double2*>(psi), reinterpret_cast<const double2*>(f),
                     reinterpret_cast<double2*>(sigma), reinterpret_cast<double2*>(theta), reinterpret_cast<double2*>(f2),
                     static_cast<hipStream_t>(stream));
}

extern "C" smg_status smg_acceleration(smg_plan* p, const double* phi, const double* theta, double* g_a, double* g_b,
                                       double* g_phi, void* stream) {
  STCHK(need_ready(p));
  if (!phi || !g_a || !g_b || !g_phi) return fail(SMG_EINVAL, "phi and the three face arrays must not be NULL");
  const double2* th = theta ? reinterpret_cast<const double2*>(theta) : (p->have_theta ? p->dptr(p->w_theta) : nullptr);
  if (!th) return fail(SMG_ESTATE, "no ghost potential yet: pass theta or call smg_solve first");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Spec& s = p->spec;
  const char* base = p->ws + p->w_blob;
  double* gpot = reinterpret_cast<double*>(p->ws + p->w_gpot);
  const double2* tw = reinterpret_cast<const double2*>(base + p->o_tw);
  HIPCHK(smgk::fft_c2r(th, gpot, p->n_g, s.n_phi, tw, st));
  AccelArgs a{};
  a.phi = phi;
  a.gpot = gpot;
  a.inv_da = reinterpret_cast<const double*>(base + p->o_acc_da);
  a.inv_db = reinterpret_cast<const double*>(base + p->o_acc_db);
  a.inv_ra = reinterpret_cast<const double*>(base + p->o_acc_ra);
  a.inv_sb = reinterpret_cast<const double*>(base + p->o_acc_sb);
  a.ga = g_a;
  a.gb = g_b;
  a.gp = g_phi;
  a.na = s.n_a;
  a.nb = s.n_b;
  a.nphi = s.n_phi;
  a.inv_dphi = 1.0 / s.dphi();
  a.sph = s.sph() ? 1 : 0;
  a.g_ahi = p->acc_g_ahi;
  a.g_blo = p->acc_g_blo;
  a.g_bhi = p->acc_g_bhi;
  HIPCHK(smgk::accel(a, st));
  return SMG_OK;
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

extern "C" const char* smg_tune_report(const smg_plan* p) { return p ? p->tune_report.c_str() : ""; }

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
