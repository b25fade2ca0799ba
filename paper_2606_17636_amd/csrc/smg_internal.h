// Internal declarations of the smg library: host plan tables and the device
// launchers.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/smg.h"

namespace smg {

enum EdgeKind { EDGE_DIRICHLET = 0, EDGE_POLE = 1, EDGE_NEUMANN = 2 };

// Grid description in host form.
struct Spec {
  int geometry, radial, n_a, n_b, n_phi;
  double a_min, a_max, b_min, b_max, G;
  bool sph() const { return geometry == SMG_SPHERICAL; }
  bool pole_lo() const;
  bool pole_hi() const;
  int n_modes() const { return n_phi / 2 + 1; }
  double dphi() const;
  double radial_face(double f) const;  // fine face index -> coordinate
  double b_face(long f) const;         // fine face index -> coordinate (pole exact)
  bool b_face_is_pole(long f) const;
};

// One axis of one level: interior cells 1..n; faces at law(off + (q-1)*stride)
// for q = 0..n+2 (q = 0 and n+2 are the ghost faces).
struct Axis {
  char which;  // 'a' radial, 'b' theta / z
  int n;
  long off, stride;
  bool pole_lo = false, pole_hi = false;
  std::vector<double> face;  // n+3
  std::vector<double> sinf;  // n+3, spherical theta only (0 at poles)
  std::vector<double> cent;  // n+2 (0 and n+1 are ghosts)
  std::vector<double> vol;   // n+2
  std::vector<double> up, dn;  // n+2: coupling of local cell k to k+1 / k-1
  std::vector<double> R;       // n+2: spherical radial metric factor R_k (1 otherwise)
  std::vector<double> P;       // n+2: factor of -s_m^2 in the azimuthal eigenvalue
};

Axis make_axis(const Spec& s, char which, long off, long stride, int n);

// Host tables of one multigrid level (main grid or DGF extended box).
struct LevelTables {
  int na, nb;
  int edge[4];  // a_lo, a_hi, b_lo, b_hi
  double dk[4]; // ghost factor of Dirichlet edges (0 on the finest level)
  Axis A, B;
  // interior arrays (length na or nb), ghost couplings removed
  std::vector<double> ua, da, Rr, ub, db;
  std::vector<double> Ca, Cb;   // [M][na], [M][nb]; diag c = Ca[i] + Rr[i] * Cb[j]
  std::vector<double> wr, wb;   // [M][nb] radial-line omega, [M][na] polar-line omega
  std::vector<double> wc;       // [M] coarsest red-black omega
  // coarsest level: fast-diagonalisation factors per mode (else empty)
  std::vector<double> sep_v;    // [M][nb][nb] at [q][j]: V[j][q], eigenvectors of the b operator
  std::vector<double> sep_vi;   // [M][nb][nb] at [j][q]: V^-1[q][j]
  std::vector<double> sep_cp;   // [M][na][nb] Thomas upper factor of (A + lambda_q Rr) at [i][q]
  std::vector<double> sep_id;   // [M][na][nb] inverse pivots, [i][q]
  std::vector<double> va, vb;   // normalised volume weights (sum_ij va_i vb_j = 1)
  // restriction to the next coarser level: [nc][2]
  std::vector<double> rwa, rwb;
  // prolongation from the next coarser level: per fine index two coarse
  // indices and weights (ghosts folded with kappa); b tables for even/odd m
  std::vector<int> pa_i0, pa_i1;
  std::vector<double> pa_w0, pa_w1;
  std::vector<int> pb_i0[2], pb_i1[2];
  std::vector<double> pb_w0[2], pb_w1[2];
};

struct Hierarchy {
  Spec spec;
  int M;  // number of mode indices the tables cover
  std::vector<LevelTables> lv;
  const char* stop = "";  // why coarsening stopped at the last level
};

// Build a hierarchy for interior cells a in [a_lo, a_lo + na - 1] and b in
// [b_lo, b_lo + nb - 1] (global fine indices) with the given edge kinds.
// `modes` is the list of azimuthal indices tables are built for (index into
// the per-mode tables = position in the list).
void separable_factors(LevelTables& T, int M);
// max_coarse: coarsening stops at the first level with at most this many
// cells (after at least one halving); 0 takes kMaxDirect.
// exact_coarse: build the fast-diagonalisation factors of the coarsest
// level (otherwise it is solved by red-black SOR).
Hierarchy build_hierarchy(const Spec& s, long a_lo, int na, long b_lo, int nb, const int edge[4],
                          const std::vector<int>& modes, bool main_grid, int max_coarse = 0,
                          bool exact_coarse = true);

// Coarsest levels up to this many cells are solved with a precomputed
// inverse instead of red-black SOR.
constexpr int kMaxDirect = 128;

double mode_s2(int n_phi, int m);
double kappa(int kind, int m);

// The Dirichlet ghost cells of the problem grid (order: inner radial j=1..nb,
// outer radial, lower b i=1..na, upper b; pole edges have none).
struct GhostSet {
  int n = 0;
  std::vector<int> gi, gj;        // global fine indices (0 / n+1 on the ghost side)
  std::vector<int> edge;          // 0 a_lo, 1 a_hi, 2 b_lo, 3 b_hi
  std::vector<double> a, b, dv3;  // centroid coordinates, 3D volume
  std::vector<double> coup_out;   // ghost -> interior coupling (screening mass)
  std::vector<double> coup_in;    // interior -> ghost coupling (boundary data)
  std::vector<int> adj;           // interior cell index i*nb + j (0-based)
};
GhostSet make_ghosts(const Spec& s);

std::string strprintf(const char* fmt, ...);

}  // namespace smg

// ---------------------------------------------------------------------------
// Device-side views and launchers (implemented in the .hip files).
// ---------------------------------------------------------------------------
struct LevelDev {
  int na, nb;
  int M;                     // per-mode table stride
  const double *ua, *da, *Rr, *ub, *db;
  const double *Ca, *Cb;     // [M][na], [M][nb]
  const double *wr, *wb, *wc;
  const double *va, *vb;
  const double *rwa, *rwb;   // restriction to the next level
  const int *pa_i0, *pa_i1;  // prolongation from the next level
  const double *pa_w0, *pa_w1;
  const int *pb_i0, *pb_i1;  // [2][nb]
  const double *pb_w0, *pb_w1;
  const double *sep_v, *sep_vi, *sep_cp, *sep_id;  // coarsest fast-diagonalisation factors, or nullptr
};

// The levels that one block per plane processes entirely in LDS (the
// coarse end of the V-cycle); L[0] is the first fused level.
constexpr int kMaxLdsLevels = 8;
struct LdsLevels {
  int n;
  int alias;    // 1: the coarser levels share LDS with the first level's f (reloaded after them)
  int scratch;  // words of exact-line scratch (0 for the SOR smoother)
  LevelDev L[kMaxLdsLevels];
};

// ---------------------------------------------------------------------------
// Batched launches.  A launch covers a list of planes of one or several
// problems (plans).  Entry e of the list packs (problem << kSlotBits | slot);
// the list and, optionally, its length live in device memory so that the
// convergence test can shrink it on the device between V-cycles.  The grid
// is sized for `cap` planes; blocks beyond the device count return at once.
// ---------------------------------------------------------------------------
constexpr int kSlotBits = 20;
__host__ __device__ inline int ent_prob(int e) { return e >> kSlotBits; }
__host__ __device__ inline int ent_slot(int e) { return e & ((1 << kSlotBits) - 1); }
__host__ __device__ inline int ent_make(int prob, int slot) { return (prob << kSlotBits) | slot; }

struct BatchRef {
  int cap;           // planes the grid is sized for
  const int* count;  // device list length (nullptr: cap)
  const int* ent;    // device list
};

// One problem's view of one multigrid depth: the tables of this level and of
// the next coarser one, the level arrays (double2 or float2, as the kernel's
// real type says) and the smoother's launch shape per line direction
// (0 radial lines, 1 polar lines).
struct LvJob {
  LevelDev L, C;
  void *u, *f, *uc, *fc;
  void* u2;          // second iterate array of the level: radial-line launches
                     // read u and write u2, polar-line launches read u2 and
                     // write u, so no block reads lines another block of the
                     // same launch writes
  double2* acc;      // mixed form, finest level: the FP64 iterate (else nullptr)
  const int* mode;   // azimuthal index of each slot (nullptr: the slot itself)
  int active;        // 0: this problem's V-cycle is fused in LDS from this depth on
  int tile[2];       // lines per block
  int ntile[2];      // blocks per plane
  int scratch[2];    // exact-line scratch words
};

// One problem's fused coarse end of the V-cycle (mg_lds.hip).
constexpr int kLdsLayoutSlots = 3 * kMaxLdsLevels + 5;
struct LdsJob {
  LdsLevels LL;
  int off[kLdsLayoutSlots];  // LDS byte offsets of the cycle's arrays (smgk::lds_cycle_layout)
  void* u;           // first fused level arrays (R typed; the coarsest is FP64)
  const void* f;
  const int* mode;
  int load_u;        // the first fused level is the finest: u holds the iterate
};

// One problem's finest level for the defect norms, the FP64 accumulation of
// the mixed form and the convergence state.
struct NormJob {
  LevelDev L;
  double2* u;        // FP64 iterate
  const double2* f;  // FP64 right-hand side
  float2 *r32, *e32; // mixed form: FP32 residual and correction (else nullptr)
  const int* mode;
  int base;          // global index of slot 0 in the convergence state arrays
};

// Per-plane convergence state, indexed by global plane index.
struct ConvState {
  double *d0, *thr, *cur;
  int* cyc;
};

// Face acceleration (accel.hip): g = -grad Phi on every cell face of the
// real potential, the boundary faces from the ghost potential.
struct AccelArgs {
  const double* phi;     // [na][nb][nphi] potential
  const double* gpot;    // [n_g][nphi] minus the ghost potential (the c2r transform of Theta)
  const double* inv_da;  // [na + 1] 1 / (centroid distance) across the radial faces 0..na
  const double* inv_db;  // [nb + 1] the same across the theta / z faces (0 on a face lying on a pole)
  const double* inv_ra;  // [na] 1 / radial centroid (theta-face and phi-face metric)
  const double* inv_sb;  // [nb] 1 / sin(theta centroid) (1 for cylindrical grids)
  double *ga, *gb, *gp;  // [na + 1][nb][nphi], [na][nb + 1][nphi], [na][nb][nphi]
  int na, nb, nphi;
  double inv_dphi;
  int sph;               // theta-face distance carries the radial centroid
  int g_ahi, g_blo, g_bhi;  // first ghost of the outer radial / lower b / upper b edge (-1: none)
};

namespace smgk {
// Face acceleration (accel.hip)
hipError_t accel(const AccelArgs& a, hipStream_t st);
// FFT (fft.hip)
// modes2 (optional): a second array given the same values (the plan's
// solve-2 right-hand side, which the James steps then complete in place).
hipError_t fft_r2c(const double* rho, double2* modes, int n_lines, int n_phi, double scale,
                   const double2* tw, hipStream_t st, double2* modes2 = nullptr);
hipError_t fft_c2r(const double2* modes, double* out, int n_lines, int n_phi, const double2* tw,
                   hipStream_t st);
// Multigrid (mg.hip).  `jobs` is the device array of one depth's LvJob per
// problem, `hj` its host mirror (used only to size the grid and LDS).
// The next smoother launch on this host thread records its start and stop
// on these events (hipExtLaunchKernelGGL: the dispatch's own timestamps, no
// event commands around the launch); one launch consumes them.
void next_launch_events(hipEvent_t start, hipEvent_t stop);
// With prolong set (radial lines, dir 0, only) the launch first adds the
// prolonged coarse correction (the job's uc) to u, in place of an
// mg_prolong launch.  With accumulate set (polar lines, dir 1, FP32 only)
// the relaxed correction of the owned lines is added to the job's FP64
// iterate (acc) instead of being stored to u, in place of an mg_accumulate
// launch.  With zero set (radial lines) the launch takes u = 0 instead of
// reading it (the first launch of a correction cycle that starts from zero).
hipError_t mg_smooth_dir(const LvJob* jobs, const LvJob* hj, int n_prob, const BatchRef& b, int n_sor, bool exact,
                         int dir, bool fp32, hipStream_t st, bool prolong = false, bool accumulate = false,
                         bool zero = false);
hipError_t mg_restrict(const LvJob* jobs, const LvJob* hj, int n_prob, const BatchRef& b, bool fp32, hipStream_t st);
hipError_t mg_prolong(const LvJob* jobs, const LvJob* hj, int n_prob, const BatchRef& b, bool fp32, hipStream_t st);
hipError_t mg_residual(const LvJob* jobs, const LvJob* hj, int n_prob, const BatchRef& b, double2* r, hipStream_t st);
// Largest dynamic LDS allocation of one block on the current device.
size_t lds_limit();
// Launch shape of the smoother for a level seen by `planes` planes at once.
struct SmoothShape { int tile, ntile, scratch; size_t lds; };
bool smooth_shape(const LevelDev& L, int dir, bool exact, bool fp32, int target_blocks, int planes, SmoothShape* out);
// fused coarse cycle (mg_lds.hip)
size_t lds_cycle_bytes(const LdsLevels& LL, bool fp32);
// The LDS byte offsets of the fused cycle's arrays, as the kernel uses them.
void lds_cycle_layout(const LdsLevels& LL, bool fp32, int* off);
// Largest first-level f the aliased layout can restrict through registers.
bool lds_cycle_alias_ok(const LdsLevels& LL);
int lds_cycle_scratch(const LdsLevels& LL, bool exact);
int lds_cycle_threads(const LdsLevels& LL);
hipError_t mg_lds_cycle(const LdsJob* jobs, const LdsJob* hj, int n_prob, const BatchRef& b, int nu_pre, int nu_post,
                        int n_sor, bool exact, bool fp32, double rtol, int max_sweeps, hipStream_t st);
// Norms and convergence (sched.hip).  mg_norm_partial: volume-weighted
// squared defect per (list position, block); use_u = 0 takes the zero guess
// (defect = f).  With the mixed form the FP64 residual is also stored
// rounded to FP32 and the FP32 correction zeroed, unless norm_only.
int norm_blocks(const NormJob* hj, int n_prob);
hipError_t mg_norm_partial(const NormJob* jobs, const NormJob* hj, int n_prob, const BatchRef& b, bool use_u,
                           double* partial, int nblk, hipStream_t st, bool zero_e = true, bool zero_u = false,
                           bool norm_only = false);
// Thresholds from the zero-guess defects: thr = tol * max(d0, floor * max
// over the problem's planes of d0); cyc = 0; the list keeps the planes
// whose d0 exceeds thr.  The full list of n planes is `all` (n <= 4096).
hipError_t mg_conv_init(const NormJob* jobs, const int* all, int n, int n_prob, const double* partial, int nblk,
                        double tol, double floor_factor, ConvState cs, int* list, int* count, hipStream_t st);
// After a V-cycle on the first `cap` planes of the list: record their
// defect norm, count the cycle (count_cycle), and keep the planes whose norm
// is above thr and whose cycle count is below max_cycles.  Planes at list
// positions >= cap were not cycled and stay.  Compacts the list in place.
hipError_t mg_converge(const NormJob* jobs, int cap, const double* partial, int nblk, ConvState cs, int max_cycles,
                       int count_cycle, int* list, int* count, hipStream_t st);
hipError_t mg_accumulate(const NormJob* jobs, const NormJob* hj, int n_prob, const BatchRef& b, hipStream_t st);
hipError_t fill_zero(double2* p, size_t n, hipStream_t st);
hipError_t copy_planes(double2* dst, const double2* src, size_t n, hipStream_t st);
// James boundary (james.hip)
hipError_t james_screen(const int* adj, const double* coup, int n_g, int plane, int M,
                        const double2* psi, double inv4piG, double2* sigma, hipStream_t st);
hipError_t james_conv(const double* dgf, const double2* sigma, double2* theta, int n_g, int M,
                      hipStream_t st);
hipError_t james_apply(const int* cells, const int* g0, const int* g1, const double* c0,
                       const double* c1, int n_cells, int plane, int n_g, int M, const double2* theta,
                       const double2* f, double2* f2, hipStream_t st);
}  // namespace smgk
