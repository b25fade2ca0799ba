// Host driver of the batched multigrid: the per-mode solves of one or
// several problems run as one sequence of launches per V-cycle (all planes
// of all problems in each launch), with the convergence test and the list of
// planes still cycling kept on the device.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "smg.h"
#include "smg_internal.h"

namespace smg {

// One problem as the engine sees it.
struct MGProblem {
  std::vector<LevelDev> L;         // level views (device tables)
  std::vector<void*> u, f;         // per-level cycle arrays; level 0 only for the mixed form (FP32)
  std::vector<void*> u2;           // per-level second iterate array of the smoother (level 0: the
                                   // cycle's type, shared by the targets)
  // a target is one solve: its FP64 iterate and right-hand side arrays
  std::vector<double2*> u0;
  std::vector<const double2*> f0;
  float2 *r32 = nullptr, *e32 = nullptr;  // mixed form: FP32 residual / correction (= f[0], u[0])
  const int* mode = nullptr;       // device azimuthal index per slot (nullptr: the slot)
  int n = 0;                       // planes
};

struct MGParams {
  int nu_pre = 2, nu_post = 2, n_sor = 2;
  bool exact = false, fp32 = false;
  double coarse_rtol = 1e-10;
  int coarse_sweeps = 1000;
};

// Launch configuration used for V-cycles over at most `cap_hi` planes.
struct MGConfig {
  int cap_hi = 0;
  int target_blocks = 512;
  std::vector<int> lds_first;  // per problem
};

// Optional per-launch event timing.
struct ProfSink {
  virtual ~ProfSink() = default;
  virtual int mark(hipStream_t st) = 0;
  virtual void close(int cls, int ev, double bytes, hipStream_t st) = 0;
  // An unrecorded event pair for a launch that records its own start and
  // stop (the dispatch's timestamps; smgk::next_launch_events): returns an
  // id for close_launch, or -1 when the sink has none.
  virtual int launch_events(hipEvent_t* start, hipEvent_t* stop) { (void)start; (void)stop; return -1; }
  virtual void close_launch(int cls, int id, double bytes) { (void)cls; (void)id; (void)bytes; }
};
enum EngineClass {
  EC_SMOOTH_R0, EC_SMOOTH_P0, EC_SMOOTH_RC, EC_SMOOTH_PC, EC_RESTRICT, EC_PROLONG, EC_COARSE, EC_NORM, EC_ACCUM, EC_CONV
};

class Engine {
 public:
  static constexpr int kMaxConfigs = 6;
  static constexpr int kNormBlocks = 64;
  static constexpr int kMaxPlanes = 4096;

  // Device bytes the engine carves from its region.
  static size_t region_bytes(int n_targets, int n_prob, int max_levels, int n_planes);

  // Sets up tables for `probs` (every problem must have the same number of
  // targets); uploads them to `region` on st and synchronises.
  smg_status init(std::vector<MGProblem> probs, int n_targets, const MGParams& prm, char* region, size_t bytes,
                  hipStream_t st, std::string* err);

  int n_planes() const { return n_total_; }
  int n_prob() const { return (int)P_.size(); }
  int base(int q) const { return base_[q]; }  // global index of problem q's first plane
  const MGParams& params() const { return prm_; }
  const std::vector<MGConfig>& configs() const { return cfg_; }
  // Replace the configurations (the last one must cover every plane).
  smg_status set_configs(const std::vector<MGConfig>& c, hipStream_t st, std::string* err);
  MGConfig default_config(int target_blocks) const;
  int min_lds_first(int q) const { return first_min_[q]; }
  int n_levels(int q) const { return (int)P_[q].L.size(); }

  // Enqueue on st (no host synchronisation):
  //   start:  zero-guess defects, thresholds and the list; warm = the target's
  //           u0 holds the initial guess (else the caller has zeroed it)
  //   cycle:  one V-cycle on the first `cap` listed planes, the mixed form's
  //           FP64 accumulation, their defects and the list update
  smg_status start(int target, double tol, double floor_factor, bool warm, int max_cycles, hipStream_t st);
  smg_status cycle(int target, int cap, hipStream_t st);
  // One V-cycle on the first `cap` planes of the full list (no list, no
  // norms): the V-cycle alone.  Used by the autotuner and the step API.
  smg_status vcycle_all(int target, int cap, int cfg, hipStream_t st);
  smg_status smooth_all(int target, hipStream_t st);             // one smoothing step, finest level, all planes
  smg_status residual_all(int target, double2* r, hipStream_t st);  // FP64 residual, finest level, all planes
  // Host reads (synchronise st).
  smg_status read_count(int target, hipStream_t st, int* n);
  // Both targets' list lengths with one synchronisation (n[0..T)).
  smg_status read_counts(hipStream_t st, int* n);
  smg_status read_state(int target, hipStream_t st, std::vector<int>& cyc, std::vector<double>& cur, std::vector<double>& thr,
                        std::vector<double>& d0);
  // Every target's list length and per-plane state with one synchronisation.
  struct State {
    std::vector<int> count;
    std::vector<std::vector<int>> cyc;
    std::vector<std::vector<double>> cur, thr, d0;
  };
  smg_status read_all(hipStream_t st, State* out);
  // Cycle until the list is empty, reading the count after every cycle.
  smg_status finish_dynamic(int target, hipStream_t st, int* cycles_run);
  // Time candidate configurations and keep the fastest per planes bucket.
  smg_status autotune(int target, hipStream_t st, std::string* report);

  void set_prof(ProfSink* p) { prof_ = p; }
  int max_cycles() const { return max_cycles_; }
  int n_targets() const { return T_; }

  ~Engine();

 private:
  smg_status build_jobs(int target, const MGConfig& c, std::vector<LvJob>& lv, std::vector<LdsJob>& lds);
  // accumulated: mixed form only; when non-null the cycle may end by adding
  // its correction to the FP64 iterate and reports whether it did
  smg_status vcycle(int target, int c, const BatchRef& b, hipStream_t st, bool* accumulated = nullptr);
  int config_for(int cap) const;
  int depth_of(const MGConfig& c) const;

  std::vector<MGProblem> P_;
  MGParams prm_;
  int T_ = 1;
  int n_total_ = 0;
  int Dmax_ = 0;                   // max levels over problems
  std::vector<int> base_;          // global plane index of each problem's slot 0
  std::vector<int> first_min_;     // finest feasible fused level per problem
  std::vector<MGConfig> cfg_;
  // device region
  int* d_all_ = nullptr;
  std::vector<int*> d_list_;       // per target: planes still cycling
  int* d_count_ = nullptr;         // [T] list lengths
  // mixed form whose every cycle starts with a finest-level radial launch:
  // that launch takes e = 0 itself, so the norms need not zero e
  bool zero_first_ = false;
  double* d_partial_ = nullptr;
  std::vector<ConvState> cs_;      // per target
  NormJob* d_norm_ = nullptr;      // [T][P]
  LvJob* d_lv_ = nullptr;          // [T][kMaxConfigs][Dmax][P]
  LdsJob* d_lds_ = nullptr;        // [T][kMaxConfigs][P]
  // host mirrors
  std::vector<NormJob> h_norm_;
  std::vector<LvJob> h_lv_;
  std::vector<LdsJob> h_lds_;
  int* h_pin_ = nullptr;           // pinned count readback
  char* h_state_ = nullptr;        // pinned state readback (read_all)
  size_t state_span_ = 0;          // bytes from d_count_ to the end of the last target's state
  int nblk_ = 1;
  int max_cycles_ = 60;
  int fp32_owner_ = -1;            // target whose residual the FP32 arrays hold (mixed form)
  ProfSink* prof_ = nullptr;
};

}  // namespace smg
