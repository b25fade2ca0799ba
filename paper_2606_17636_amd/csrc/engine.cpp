// Batched multigrid driver (see engine.h).
#include "engine.h"

#include <algorithm>
#include <cstring>

namespace smg {

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// One-block-per-plane fused levels of problem `P` from level `first` down:
// the plain LDS layout when it fits in 64 KiB, else the aliased one (the
// coarser levels reuse the first level's f storage).
LdsLevels lds_levels(const MGProblem& P, int first, bool exact, bool fp32) {
  LdsLevels LL{};
  const int L = (int)P.L.size();
  LL.n = L - first;
  for (int l = first; l < L; ++l) LL.L[l - first] = P.L[l];
  LL.scratch = smgk::lds_cycle_scratch(LL, exact);
  LL.alias = 0;
  if (LL.n > 1 && smgk::lds_cycle_bytes(LL, fp32) > 64 * 1024) {
    LL.alias = 1;
    if (!smgk::lds_cycle_alias_ok(LL)) LL.alias = 0;
  }
  return LL;
}

// LDS a fused-cycle block may use (the device limit less the kernel's own
// static arrays).
size_t lds_cycle_max() { return smgk::lds_limit() - 1024; }

}  // namespace

#define EHIP(expr)                                                              \
  do {                                                                          \
    hipError_t e_ = (expr);                                                     \
    if (e_ != hipSuccess) {                                                     \
      if (err) *err = strprintf("%s: %s", #expr, hipGetErrorString(e_));        \
      return SMG_EHIP;                                                          \
    }                                                                           \
  } while (0)
#define EFAIL(code, msg)       \
  do {                         \
    if (err) *err = (msg);     \
    return (code);             \
  } while (0)

size_t Engine::region_bytes(int n_targets, int n_prob, int max_levels, int n_planes) {
  size_t b = 0;
  b += (1 + n_targets) * align_up(sizeof(int) * n_planes) + align_up(sizeof(int) * n_targets);
  b += align_up(sizeof(double) * (size_t)n_planes * kNormBlocks);
  b += n_targets * (3 * align_up(sizeof(double) * n_planes) + align_up(sizeof(int) * n_planes));
  b += align_up(sizeof(NormJob) * n_targets * n_prob);
  b += align_up(sizeof(LvJob) * (size_t)n_targets * kMaxConfigs * max_levels * n_prob);
  b += align_up(sizeof(LdsJob) * (size_t)n_targets * kMaxConfigs * n_prob);
  return b;
}

Engine::~Engine() {
  if (h_pin_) (void)hipHostFree(h_pin_);
  if (h_state_) (void)hipHostFree(h_state_);
}

smg_status Engine::init(std::vector<MGProblem> probs, int n_targets, const MGParams& prm, char* region, size_t bytes,
                        hipStream_t st, std::string* err) {
  P_ = std::move(probs);
  prm_ = prm;
  T_ = n_targets;
  const int P = (int)P_.size();
  if (P < 1 || P > 256) EFAIL(SMG_EINVAL, "a batch holds 1 to 256 problems");
  base_.assign(P, 0);
  first_min_.assign(P, 0);
  n_total_ = 0;
  Dmax_ = 0;
  for (int q = 0; q < P; ++q) {
    const MGProblem& pr = P_[q];
    if (pr.L.empty() || (int)pr.u0.size() != T_ || (int)pr.f0.size() != T_ || pr.n < 1) EFAIL(SMG_EINVAL, "engine: malformed problem");
    if ((int)pr.u.size() != (int)pr.L.size() || (int)pr.f.size() != (int)pr.L.size() ||
        (int)pr.u2.size() != (int)pr.L.size())
      EFAIL(SMG_EINVAL, "engine: level arrays");
    if (prm_.fp32 && (!pr.r32 || !pr.e32)) EFAIL(SMG_EINVAL, "engine: mixed form needs FP32 residual/correction arrays");
    base_[q] = n_total_;
    n_total_ += pr.n;
    Dmax_ = std::max(Dmax_, (int)pr.L.size());
    const int L = (int)pr.L.size();
    int fm = L - 1;
    for (int first = 0; first < L; ++first) {
      if (L - first > kMaxLdsLevels) continue;
      LdsLevels LL = lds_levels(pr, first, prm_.exact, prm_.fp32);
      if (smgk::lds_cycle_bytes(LL, prm_.fp32) <= lds_cycle_max()) { fm = first; break; }
    }
    if (L - fm > kMaxLdsLevels) EFAIL(SMG_EINVAL, "engine: too many fused levels");
    LdsLevels LL = lds_levels(pr, fm, prm_.exact, prm_.fp32);
    if (smgk::lds_cycle_bytes(LL, prm_.fp32) > lds_cycle_max()) EFAIL(SMG_EINVAL, "engine: coarsest level does not fit in LDS");
    first_min_[q] = fm;
  }
  if (n_total_ > kMaxPlanes) EFAIL(SMG_EINVAL, strprintf("a batch holds at most %d planes", kMaxPlanes));
  // smoothing steps left to the engine (negative): one each way when every
  // problem smooths its finest level in whole-grid launches, where a step is
  // two latency-bound launches and fewer steps with more cycles is faster;
  // two when the whole V-cycle fits the fused kernel
  bool split = true;
  for (int q = 0; q < P; ++q)
    if (first_min_[q] == 0) split = false;
  if (prm_.nu_pre < 0) prm_.nu_pre = split ? 1 : 2;
  if (prm_.nu_post < 0) prm_.nu_post = split ? 1 : 2;
  // every configuration then smooths the finest level first (lds_first >= 1)
  zero_first_ = prm_.fp32 && split && prm_.nu_pre >= 1;
  if (bytes < region_bytes(T_, P, Dmax_, n_total_)) EFAIL(SMG_EWORKSPACE, "engine region too small");
  // carve the region
  char* q0 = region;
  auto take = [&](size_t b) { char* r = q0; q0 += align_up(b); return r; };
  d_all_ = reinterpret_cast<int*>(take(sizeof(int) * n_total_));
  d_list_.assign(T_, nullptr);
  cs_.assign(T_, ConvState{});
  for (int t = 0; t < T_; ++t) d_list_[t] = reinterpret_cast<int*>(take(sizeof(int) * n_total_));
  // the list lengths and every target's convergence state form one span,
  // which read_all copies to the host at once
  d_count_ = reinterpret_cast<int*>(take(sizeof(int) * T_));
  for (int t = 0; t < T_; ++t) {
    cs_[t].d0 = reinterpret_cast<double*>(take(sizeof(double) * n_total_));
    cs_[t].thr = reinterpret_cast<double*>(take(sizeof(double) * n_total_));
    cs_[t].cur = reinterpret_cast<double*>(take(sizeof(double) * n_total_));
    cs_[t].cyc = reinterpret_cast<int*>(take(sizeof(int) * n_total_));
  }
  state_span_ = (size_t)(reinterpret_cast<char*>(cs_[T_ - 1].cyc + n_total_) - reinterpret_cast<char*>(d_count_));
  d_partial_ = reinterpret_cast<double*>(take(sizeof(double) * (size_t)n_total_ * kNormBlocks));
  d_norm_ = reinterpret_cast<NormJob*>(take(sizeof(NormJob) * T_ * P));
  d_lv_ = reinterpret_cast<LvJob*>(take(sizeof(LvJob) * (size_t)T_ * kMaxConfigs * Dmax_ * P));
  d_lds_ = reinterpret_cast<LdsJob*>(take(sizeof(LdsJob) * (size_t)T_ * kMaxConfigs * P));
  // static lists and norm jobs
  std::vector<int> all;
  for (int q = 0; q < P; ++q)
    for (int s = 0; s < P_[q].n; ++s) all.push_back(ent_make(q, s));
  h_norm_.assign((size_t)T_ * P, NormJob{});
  for (int t = 0; t < T_; ++t)
    for (int q = 0; q < P; ++q) {
      NormJob& J = h_norm_[(size_t)t * P + q];
      J.L = P_[q].L[0];
      J.u = P_[q].u0[t];
      J.f = P_[q].f0[t];
      J.r32 = prm_.fp32 ? P_[q].r32 : nullptr;
      J.e32 = prm_.fp32 ? P_[q].e32 : nullptr;
      J.mode = P_[q].mode;
      J.base = base_[q];
    }
  nblk_ = smgk::norm_blocks(h_norm_.data(), P);
  h_lv_.assign((size_t)T_ * kMaxConfigs * Dmax_ * P, LvJob{});
  h_lds_.assign((size_t)T_ * kMaxConfigs * P, LdsJob{});
  if (!h_pin_) EHIP(hipHostMalloc((void**)&h_pin_, sizeof(int) * (kMaxPlanes + 16)));
  if (h_state_) (void)hipHostFree(h_state_);
  h_state_ = nullptr;
  EHIP(hipHostMalloc((void**)&h_state_, state_span_));
  EHIP(hipMemcpyAsync(d_all_, all.data(), sizeof(int) * all.size(), hipMemcpyHostToDevice, st));
  EHIP(hipMemcpyAsync(d_norm_, h_norm_.data(), sizeof(NormJob) * h_norm_.size(), hipMemcpyHostToDevice, st));
  // scratch configuration (last slot): every level smoothable, nothing fused;
  // serves the step-level entry points
  {
    MGConfig c;
    c.cap_hi = n_total_;
    c.target_blocks = 512;
    for (int q = 0; q < P; ++q) c.lds_first.push_back((int)P_[q].L.size());
    std::vector<LvJob> lv;
    std::vector<LdsJob> lds;
    for (int t = 0; t < T_; ++t) {
      smg_status s = build_jobs(t, c, lv, lds);
      if (s != SMG_OK) EFAIL(s, "engine: step configuration does not fit");
      std::copy(lv.begin(), lv.end(), h_lv_.begin() + ((size_t)t * kMaxConfigs + kMaxConfigs - 1) * Dmax_ * P);
    }
  }
  std::vector<MGConfig> cs{default_config(512)};
  smg_status s = set_configs(cs, st, err);
  if (s != SMG_OK) return s;
  EHIP(hipStreamSynchronize(st));
  return SMG_OK;
}

MGConfig Engine::default_config(int target_blocks) const {
  MGConfig c;
  c.cap_hi = n_total_;
  c.target_blocks = target_blocks;
  c.lds_first = first_min_;
  return c;
}

smg_status Engine::build_jobs(int target, const MGConfig& c, std::vector<LvJob>& lv, std::vector<LdsJob>& lds) {
  const int P = (int)P_.size();
  lv.assign((size_t)Dmax_ * P, LvJob{});
  lds.assign(P, LdsJob{});
  const int planes = std::max(1, std::min(c.cap_hi, n_total_));
  for (int q = 0; q < P; ++q) {
    const MGProblem& pr = P_[q];
    const int L = (int)pr.L.size();
    const int first = c.lds_first[q];
    for (int d = 0; d < L && d < Dmax_; ++d) {
      LvJob& J = lv[(size_t)d * P + q];
      J.L = pr.L[d];
      J.C = d + 1 < L ? pr.L[d + 1] : pr.L[d];
      J.u = d == 0 && !prm_.fp32 ? (void*)pr.u0[target] : pr.u[d];
      J.f = d == 0 && !prm_.fp32 ? (void*)pr.f0[target] : pr.f[d];
      J.uc = d + 1 < L ? pr.u[d + 1] : nullptr;
      J.acc = d == 0 && prm_.fp32 ? pr.u0[target] : nullptr;
      J.u2 = pr.u2[d];
      J.fc = d + 1 < L ? pr.f[d + 1] : nullptr;
      J.mode = pr.mode;
      J.active = d < first ? 1 : 0;
      for (int dir = 0; dir < 2; ++dir) {
        smgk::SmoothShape sh{};
        if (!smgk::smooth_shape(pr.L[d], dir, prm_.exact, prm_.fp32, c.target_blocks, planes, &sh)) {
          if (J.active) return SMG_EINVAL;
          J.active = 0;
        }
        J.tile[dir] = sh.tile;
        J.ntile[dir] = sh.ntile;
        J.scratch[dir] = sh.scratch;
      }
    }
    if (first < L) {
      LdsJob& J = lds[q];
      J.LL = lds_levels(pr, first, prm_.exact, prm_.fp32);
      if (smgk::lds_cycle_bytes(J.LL, prm_.fp32) > lds_cycle_max()) return SMG_EINVAL;
      smgk::lds_cycle_layout(J.LL, prm_.fp32, J.off);
      J.u = first == 0 && !prm_.fp32 ? (void*)pr.u0[target] : pr.u[first];
      J.f = first == 0 && !prm_.fp32 ? (const void*)pr.f0[target] : pr.f[first];
      J.mode = pr.mode;
      J.load_u = first == 0 ? 1 : 0;
    }
  }
  return SMG_OK;
}

smg_status Engine::set_configs(const std::vector<MGConfig>& c, hipStream_t st, std::string* err) {
  if (c.empty() || (int)c.size() > kMaxConfigs - 1) EFAIL(SMG_EINVAL, "engine: bad configuration count");
  for (const MGConfig& x : c)
    if ((int)x.lds_first.size() != (int)P_.size()) EFAIL(SMG_EINVAL, "engine: configuration does not match the problems");
  cfg_ = c;
  cfg_.back().cap_hi = std::max(cfg_.back().cap_hi, n_total_);
  for (int k = 0; k < (int)cfg_.size(); ++k) {
    for (int t = 0; t < T_; ++t) {
      std::vector<LvJob> lv;
      std::vector<LdsJob> lds;
      smg_status s = build_jobs(t, cfg_[k], lv, lds);
      if (s != SMG_OK) EFAIL(s, "engine: a configuration does not fit in LDS");
      std::copy(lv.begin(), lv.end(), h_lv_.begin() + ((size_t)t * kMaxConfigs + k) * Dmax_ * P_.size());
      std::copy(lds.begin(), lds.end(), h_lds_.begin() + ((size_t)t * kMaxConfigs + k) * P_.size());
    }
  }
  EHIP(hipMemcpyAsync(d_lv_, h_lv_.data(), sizeof(LvJob) * h_lv_.size(), hipMemcpyHostToDevice, st));
  EHIP(hipMemcpyAsync(d_lds_, h_lds_.data(), sizeof(LdsJob) * h_lds_.size(), hipMemcpyHostToDevice, st));
  // the host mirrors are read by later launches' shape computations only;
  // the copies above are from pageable memory and complete before return
  EHIP(hipStreamSynchronize(st));
  return SMG_OK;
}

int Engine::config_for(int cap) const {
  for (int k = 0; k < (int)cfg_.size(); ++k)
    if (cap <= cfg_[k].cap_hi) return k;
  return (int)cfg_.size() - 1;
}

int Engine::depth_of(const MGConfig& c) const {
  int D = 0;
  for (int x : c.lds_first) D = std::max(D, x);
  return D;
}

smg_status Engine::vcycle(int target, int c, const BatchRef& b, hipStream_t st, bool* accumulated) {
  const int P = (int)P_.size();
  const MGConfig& cf = cfg_[c];
  const size_t base = ((size_t)target * kMaxConfigs + c) * Dmax_ * P;
  const LvJob* dl = d_lv_ + base;
  const LvJob* hl = h_lv_.data() + base;
  const LdsJob* dz = d_lds_ + ((size_t)target * kMaxConfigs + c) * P;
  const LdsJob* hz = h_lds_.data() + ((size_t)target * kMaxConfigs + c) * P;
  const bool f32 = prm_.fp32;
  const double vb = f32 ? 8.0 : 16.0;
  const int D = depth_of(cf);
  // algorithmic bytes of a launch: planes x cells of the problem at depth d
  auto cells = [&](int d, bool coarse_side) {
    double s = 0.0;
    for (int q = 0; q < P; ++q) {
      if (d >= (int)P_[q].L.size()) continue;
      if (!(d < cf.lds_first[q])) continue;
      const LevelDev& L = coarse_side ? hl[(size_t)d * P + q].C : hl[(size_t)d * P + q].L;
      s += (double)L.na * L.nb * std::min(P_[q].n, b.cap);
    }
    return s;
  };
  // one smoothing step at depth d; with prolong set its first launch also
  // applies the coarse-grid correction (reads the coarse correction too);
  // with acc set its last launch adds the FP32 correction to the FP64
  // iterate (reads and writes the FP64 iterate instead of storing FP32)
  auto smooth = [&](int d, bool prolong, bool acc, bool zero) -> hipError_t {
    for (int dir = 0; dir < 2; ++dir) {
      const bool pr = prolong && dir == 0, ac = acc && dir == 1, z = zero && dir == 0;
      // profiled: the smoother launch records its own start and stop
      hipEvent_t e0 = nullptr, e1 = nullptr;
      const int id = prof_ ? prof_->launch_events(&e0, &e1) : -1;
      const int ev = prof_ && id < 0 ? prof_->mark(st) : -1;
      if (id >= 0) smgk::next_launch_events(e0, e1);
      hipError_t e = smgk::mg_smooth_dir(dl + (size_t)d * P, hl + (size_t)d * P, P, b, prm_.n_sor, prm_.exact, dir,
                                         f32, st, pr, ac, z);
      smgk::next_launch_events(nullptr, nullptr);
      if (e != hipSuccess) return e;
      const int cls = d == 0 ? (dir == 0 ? EC_SMOOTH_R0 : EC_SMOOTH_P0) : (dir == 0 ? EC_SMOOTH_RC : EC_SMOOTH_PC);
      const double bytes = ((pr ? 3.25 : 3.0) * vb + (ac ? 32.0 - vb : 0.0) - (z ? vb : 0.0)) * cells(d, false);
      if (id >= 0) prof_->close_launch(cls, id, bytes);
      else if (prof_) prof_->close(cls, ev, bytes, st);
    }
    return hipSuccess;
  };
  // the mixed form's correction step u += e goes into the last launch of the
  // cycle when every problem smooths its finest level in separate launches
  bool acc_last = accumulated && f32 && D > 0 && prm_.nu_post > 0;
  for (int q = 0; q < P; ++q)
    if (!hl[q].active) acc_last = false;
  if (accumulated) *accumulated = acc_last;
  hipError_t e = hipSuccess;
  for (int d = 0; d < D; ++d) {
    for (int k = 0; k < prm_.nu_pre; ++k)
      if ((e = smooth(d, false, false, zero_first_ && d == 0 && k == 0)) != hipSuccess) return SMG_EHIP;
    const int ev = prof_ ? prof_->mark(st) : -1;
    if ((e = smgk::mg_restrict(dl + (size_t)d * P, hl + (size_t)d * P, P, b, f32, st)) != hipSuccess) return SMG_EHIP;
    if (prof_) prof_->close(EC_RESTRICT, ev, (2.0 * vb + 0.5 * vb) * cells(d, false), st);
  }
  {
    const int ev = prof_ ? prof_->mark(st) : -1;
    if ((e = smgk::mg_lds_cycle(dz, hz, P, b, prm_.nu_pre, prm_.nu_post, prm_.n_sor, prm_.exact, f32, prm_.coarse_rtol,
                                prm_.coarse_sweeps, st)) != hipSuccess)
      return SMG_EHIP;
    if (prof_) {
      double s = 0.0;
      for (int q = 0; q < P; ++q) s += (double)hz[q].LL.L[0].na * hz[q].LL.L[0].nb * std::min(P_[q].n, b.cap);
      prof_->close(EC_COARSE, ev, 2.0 * vb * s, st);
    }
  }
  for (int d = D - 1; d >= 0; --d) {
    // the first post-smoothing launch applies the coarse correction itself
    // where its tiles own at least 8 lines (so that the halo lines, which it
    // interpolates too, are at most half the tile); else a prolongation pass
    bool fuse = prm_.nu_post > 0;
    for (int q = 0; q < P; ++q) {
      const LvJob& J = hl[(size_t)d * P + q];
      if (J.active && J.tile[0] < 8) fuse = false;
    }
    if (!fuse) {
      const int ev = prof_ ? prof_->mark(st) : -1;
      if ((e = smgk::mg_prolong(dl + (size_t)d * P, hl + (size_t)d * P, P, b, f32, st)) != hipSuccess) return SMG_EHIP;
      if (prof_) prof_->close(EC_PROLONG, ev, (2.0 * vb + 0.25 * vb) * cells(d, false), st);
    }
    for (int k = 0; k < prm_.nu_post; ++k)
      if ((e = smooth(d, fuse && k == 0, acc_last && d == 0 && k == prm_.nu_post - 1, false)) != hipSuccess)
        return SMG_EHIP;
  }
  return SMG_OK;
}

smg_status Engine::start(int target, double tol, double floor_factor, bool warm, int max_cycles, hipStream_t st) {
  const int P = (int)P_.size();
  max_cycles_ = max_cycles;
  const NormJob* dn = d_norm_ + (size_t)target * P;
  const NormJob* hn = h_norm_.data() + (size_t)target * P;
  // a cold start's zero iterate is written by the zero-guess norm below; a
  // warm start needs only the norm of f from it (its own defect pass below
  // writes the FP32 residual and clears the correction)
  BatchRef ball{n_total_, nullptr, d_all_};
  int ev = prof_ ? prof_->mark(st) : -1;
  if (smgk::mg_norm_partial(dn, hn, P, ball, false, d_partial_, nblk_, st, !zero_first_, !warm, warm) != hipSuccess)
    return SMG_EHIP;
  if (smgk::mg_conv_init(dn, d_all_, n_total_, P, d_partial_, nblk_, tol, floor_factor, cs_[target], d_list_[target],
                         d_count_ + target, st) != hipSuccess)
    return SMG_EHIP;
  if (prof_) {
    double s = 0.0;
    for (int q = 0; q < P; ++q) s += (double)P_[q].n * P_[q].L[0].na * P_[q].L[0].nb;
    prof_->close(EC_NORM, ev, (prm_.fp32 && !warm ? 32.0 : 16.0) * s, st);
  }
  fp32_owner_ = target;
  if (warm) {
    BatchRef b{n_total_, d_count_ + target, d_list_[target]};
    if (smgk::mg_norm_partial(dn, hn, P, b, true, d_partial_, nblk_, st, !zero_first_) != hipSuccess) return SMG_EHIP;
    if (smgk::mg_converge(dn, n_total_, d_partial_, nblk_, cs_[target], max_cycles_, 0, d_list_[target],
                          d_count_ + target, st) != hipSuccess)
      return SMG_EHIP;
  }
  return SMG_OK;
}

smg_status Engine::cycle(int target, int cap, hipStream_t st) {
  if (cap <= 0) return SMG_OK;
  cap = std::min(cap, n_total_);
  const int P = (int)P_.size();
  const NormJob* dn = d_norm_ + (size_t)target * P;
  const NormJob* hn = h_norm_.data() + (size_t)target * P;
  BatchRef b{cap, d_count_ + target, d_list_[target]};
  if (prm_.fp32 && fp32_owner_ != target) {
    // the FP32 residual arrays (shared by the targets) hold another solve's
    // residual: recompute this target's for every listed plane
    BatchRef all{n_total_, d_count_ + target, d_list_[target]};
    if (smgk::mg_norm_partial(dn, hn, P, all, true, d_partial_, nblk_, st, !zero_first_) != hipSuccess) return SMG_EHIP;
    if (smgk::mg_converge(dn, n_total_, d_partial_, nblk_, cs_[target], max_cycles_, 0, d_list_[target],
                          d_count_ + target, st) != hipSuccess)
      return SMG_EHIP;
    fp32_owner_ = target;
  }
  bool accumulated = false;
  smg_status s = vcycle(target, config_for(cap), b, st, &accumulated);
  if (s != SMG_OK) return s;
  double cells = 0.0;
  for (int q = 0; q < P; ++q) cells += (double)std::min(P_[q].n, cap) * P_[q].L[0].na * P_[q].L[0].nb;
  if (prm_.fp32 && !accumulated) {
    const int ev = prof_ ? prof_->mark(st) : -1;
    if (smgk::mg_accumulate(dn, hn, P, b, st) != hipSuccess) return SMG_EHIP;
    if (prof_) prof_->close(EC_ACCUM, ev, 40.0 * cells, st);
  }
  const int ev = prof_ ? prof_->mark(st) : -1;
  if (smgk::mg_norm_partial(dn, hn, P, b, true, d_partial_, nblk_, st, !zero_first_) != hipSuccess) return SMG_EHIP;
  if (prof_) prof_->close(EC_NORM, ev, (prm_.fp32 ? 48.0 : 32.0) * cells, st);
  if (smgk::mg_converge(dn, cap, d_partial_, nblk_, cs_[target], max_cycles_, 1, d_list_[target], d_count_ + target,
                        st) != hipSuccess)
    return SMG_EHIP;
  return SMG_OK;
}

smg_status Engine::vcycle_all(int target, int cap, int cfg, hipStream_t st) {
  BatchRef b{std::min(cap, n_total_), nullptr, d_all_};
  return vcycle(target, cfg, b, st);
}

smg_status Engine::smooth_all(int target, hipStream_t st) {
  const int P = (int)P_.size();
  const size_t base = ((size_t)target * kMaxConfigs + kMaxConfigs - 1) * Dmax_ * P;
  BatchRef b{n_total_, nullptr, d_all_};
  for (int dir = 0; dir < 2; ++dir)
    if (smgk::mg_smooth_dir(d_lv_ + base, h_lv_.data() + base, P, b, prm_.n_sor, prm_.exact, dir, prm_.fp32, st) !=
        hipSuccess)
      return SMG_EHIP;
  return SMG_OK;
}

smg_status Engine::residual_all(int target, double2* r, hipStream_t st) {
  if (prm_.fp32) return SMG_EINVAL;
  const int P = (int)P_.size();
  const size_t base = ((size_t)target * kMaxConfigs + kMaxConfigs - 1) * Dmax_ * P;
  BatchRef b{n_total_, nullptr, d_all_};
  if (smgk::mg_residual(d_lv_ + base, h_lv_.data() + base, P, b, r, st) != hipSuccess) return SMG_EHIP;
  return SMG_OK;
}

smg_status Engine::read_count(int target, hipStream_t st, int* n) {
  if (hipMemcpyAsync(h_pin_, d_count_ + target, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess) return SMG_EHIP;
  if (hipStreamSynchronize(st) != hipSuccess) return SMG_EHIP;
  *n = h_pin_[0];
  return SMG_OK;
}

smg_status Engine::read_counts(hipStream_t st, int* n) {
  if (hipMemcpyAsync(h_pin_, d_count_, sizeof(int) * T_, hipMemcpyDeviceToHost, st) != hipSuccess) return SMG_EHIP;
  if (hipStreamSynchronize(st) != hipSuccess) return SMG_EHIP;
  for (int t = 0; t < T_; ++t) n[t] = h_pin_[t];
  return SMG_OK;
}

smg_status Engine::read_state(int target, hipStream_t st, std::vector<int>& cyc, std::vector<double>& cur,
                              std::vector<double>& thr, std::vector<double>& d0) {
  const ConvState& c = cs_[target];
  cyc.resize(n_total_);
  cur.resize(n_total_);
  thr.resize(n_total_);
  d0.resize(n_total_);
  if (hipMemcpyAsync(cyc.data(), c.cyc, sizeof(int) * n_total_, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(cur.data(), c.cur, sizeof(double) * n_total_, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(thr.data(), c.thr, sizeof(double) * n_total_, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(d0.data(), c.d0, sizeof(double) * n_total_, hipMemcpyDeviceToHost, st) != hipSuccess)
    return SMG_EHIP;
  if (hipStreamSynchronize(st) != hipSuccess) return SMG_EHIP;
  return SMG_OK;
}

smg_status Engine::read_all(hipStream_t st, State* out) {
  // one copy of the span [list lengths, every target's state]
  if (hipMemcpyAsync(h_state_, d_count_, state_span_, hipMemcpyDeviceToHost, st) != hipSuccess) return SMG_EHIP;
  if (hipStreamSynchronize(st) != hipSuccess) return SMG_EHIP;
  const size_t n = n_total_;
  const char* base = reinterpret_cast<const char*>(d_count_);
  auto host = [&](const void* dev) { return h_state_ + (reinterpret_cast<const char*>(dev) - base); };
  const int* cnt = reinterpret_cast<const int*>(h_state_);
  out->count.assign(cnt, cnt + T_);
  out->cyc.resize(T_);
  out->cur.resize(T_);
  out->thr.resize(T_);
  out->d0.resize(T_);
  for (int t = 0; t < T_; ++t) {
    const ConvState& c = cs_[t];
    const double* cur = reinterpret_cast<const double*>(host(c.cur));
    const double* thr = reinterpret_cast<const double*>(host(c.thr));
    const double* d0 = reinterpret_cast<const double*>(host(c.d0));
    const int* cyc = reinterpret_cast<const int*>(host(c.cyc));
    out->cur[t].assign(cur, cur + n);
    out->thr[t].assign(thr, thr + n);
    out->d0[t].assign(d0, d0 + n);
    out->cyc[t].assign(cyc, cyc + n);
  }
  return SMG_OK;
}

smg_status Engine::finish_dynamic(int target, hipStream_t st, int* cycles_run) {
  int runs = 0;
  for (int guard = 0; guard <= max_cycles_ + 1; ++guard) {
    int n = 0;
    smg_status s = read_count(target, st, &n);
    if (s != SMG_OK) return s;
    if (n == 0) break;
    s = cycle(target, n, st);
    if (s != SMG_OK) return s;
    ++runs;
  }
  if (cycles_run) *cycles_run = runs;
  return SMG_OK;
}

smg_status Engine::autotune(int target, hipStream_t st, std::string* report) {
  std::string* err = report;
  const int P = (int)P_.size();
  // plane-count buckets; a launch takes the configuration of the first
  // bucket that holds its planes
  std::vector<int> caps;
  for (int c : {2, 8, 32}) if (c < n_total_) caps.push_back(c);
  caps.push_back(n_total_);
  hipEvent_t e0, e1;
  EHIP(hipEventCreate(&e0));
  EHIP(hipEventCreate(&e1));
  struct Guard { hipEvent_t a, b; ~Guard() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); } } g{e0, e1};
  std::vector<MGConfig> best;
  std::string rep;
  const int scratch = kMaxConfigs - 2;
  // Within a bucket the first candidate (in the order tried: fused range
  // from the finest feasible level, then fewer blocks) whose time is within
  // kTuneTie of the fastest is kept, so that near-equal candidates do not
  // trade places from one process to the next on timing noise.
  constexpr float kTuneTie = 1.03f;
  for (size_t ci = 0; ci < caps.size(); ++ci) {
    const int cap = caps[ci];
    // a bucket serves every launch of (lo, cap] planes: candidates are timed
    // at its top, middle and bottom plane counts, since a shape that fills
    // the device exactly at the top can leave a partly filled last round of
    // blocks below it
    const int lo = ci > 0 ? caps[ci - 1] : 0;
    std::vector<int> counts{cap};
    const int mid = lo + (cap - lo + 1) / 2;
    if (mid > lo && mid < cap) counts.push_back(mid);
    if (lo + 1 < cap && lo + 1 != mid) counts.push_back(lo + 1);
    std::vector<std::pair<MGConfig, float>> cand;
    for (int off = 0; off < 3; ++off) {
      bool any_new = false;
      MGConfig c;
      c.cap_hi = cap;
      for (int q = 0; q < P; ++q) {
        const int f = std::min(first_min_[q] + off, (int)P_[q].L.size() - 1);
        c.lds_first.push_back(f);
        if (first_min_[q] + off <= (int)P_[q].L.size() - 1) any_new = true;
      }
      if (off > 0 && !any_new) break;
      for (int tb : {256, 384, 512, 768, 1024, 1536, 2048, 3072, 4096}) {
        c.target_blocks = tb;
        // stage the candidate in the scratch slot
        std::vector<LvJob> lv;
        std::vector<LdsJob> lds;
        if (build_jobs(target, c, lv, lds) != SMG_OK) continue;
        std::copy(lv.begin(), lv.end(), h_lv_.begin() + ((size_t)target * kMaxConfigs + scratch) * Dmax_ * P);
        std::copy(lds.begin(), lds.end(), h_lds_.begin() + ((size_t)target * kMaxConfigs + scratch) * P);
        EHIP(hipMemcpyAsync(d_lv_ + ((size_t)target * kMaxConfigs + scratch) * Dmax_ * P, lv.data(),
                            sizeof(LvJob) * lv.size(), hipMemcpyHostToDevice, st));
        EHIP(hipMemcpyAsync(d_lds_ + ((size_t)target * kMaxConfigs + scratch) * P, lds.data(), sizeof(LdsJob) * lds.size(),
                            hipMemcpyHostToDevice, st));
        const MGConfig keep = cfg_.size() > (size_t)scratch ? cfg_[scratch] : MGConfig{};
        if ((int)cfg_.size() <= scratch) cfg_.resize(scratch + 1, c);
        cfg_[scratch] = c;
        smg_status s = vcycle_all(target, cap, scratch, st);
        float ms = 0.f;
        for (size_t k = 0; k < counts.size() && s == SMG_OK; ++k) {
          EHIP(hipEventRecord(e0, st));
          for (int r = 0; r < 5 && s == SMG_OK; ++r) s = vcycle_all(target, counts[k], scratch, st);
          EHIP(hipEventRecord(e1, st));
          EHIP(hipEventSynchronize(e1));
          float t = 0.f;
          EHIP(hipEventElapsedTime(&t, e0, e1));
          ms += t / 5.f;
        }
        cfg_[scratch] = keep;
        if (s != SMG_OK) return s;
        rep += strprintf("planes %d..%d: fused from +%d, %d blocks: %.1f us\n", lo + 1, cap, off, tb, 1e3 * ms);
        cand.emplace_back(c, ms);
      }
    }
    if (cand.empty()) EFAIL(SMG_EINVAL, "autotune: no configuration fits");
    float bt = 1e30f;
    for (const auto& cm : cand) bt = std::min(bt, cm.second);
    MGConfig bc = cand[0].first;
    for (const auto& cm : cand)
      if (cm.second <= kTuneTie * bt) {
        bc = cm.first;
        break;
      }
    rep += strprintf("planes <= %d: fused from level %d (+%d), %d blocks\n", cap, bc.lds_first[0], bc.lds_first[0] - first_min_[0], bc.target_blocks);
    best.push_back(bc);
  }
  cfg_.resize(std::min(cfg_.size(), (size_t)scratch));
  smg_status s = set_configs(best, st, err);
  if (report) *report = rep;
  return s;
}

}  // namespace smg
