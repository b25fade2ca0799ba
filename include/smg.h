/*
 * smg.h -- C ABI of the MI355X spectral-multigrid Poisson solver.
 *
 * Solves the finite-volume Poisson equation  lap Phi = 4 pi G rho  on a
 * spherical (r, theta, phi) or cylindrical (R, phi, z) grid with uniform or
 * logarithmic radial spacing and vacuum (isolated) boundaries, following
 * Mandal, Gressel, Ziegler & Mignone, "A fast spectral-multigrid Poisson
 * solver in non-Cartesian geometries": an azimuthal real FFT (Sec. 2.2)
 * splits the problem into one 2D Helmholtz problem per Fourier mode
 * m = 0..n_phi/2 (Eqs. helmholz_sph / helmholz_cyl), each solved by
 * geometric multigrid (Sec. 3) with the James screening-mass boundary
 * (Sec. 4), then the inverse FFT returns the potential (Sec. 5.1).
 *
 * Conventions shared by every entry point
 *  - All pointers named *_dev are device (HIP) pointers owned by the caller;
 *    *_host pointers are host memory owned by the caller.  The library owns
 *    only the opaque host-side plan object.
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).  All
 *    device work of a call is enqueued on it.  Calls that return host data
 *    (info structs, *_host outputs) synchronise the stream before returning.
 *  - Real-space arrays (density, potential) are FP64, interior cells only,
 *    C order [n_a][n_b][n_phi] with phi fastest.  a = r (spherical) or R
 *    (cylindrical); b = theta (spherical) or z (cylindrical).  A cylindrical
 *    caller permutes (R, phi, z) to (R, z, phi).
 *  - Mode arrays are interleaved complex FP64 (re, im), C order
 *    [n_phi/2 + 1][n_a][n_b] with b fastest.
 *  - Every function returns an smg_status; on failure smg_last_error()
 *    returns a thread-local message.  No exception or abort crosses the ABI.
 *  - A plan and its workspace may be used by one stream at a time; calls
 *    that overlap on one plan race.
 */
#ifndef SMG_H
#define SMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SMG_OK = 0,
  SMG_EINVAL = -1,      /* invalid argument or unsupported grid            */
  SMG_ENOCONV = -2,     /* a mode missed the tolerance within max_cycles;
                           outputs hold the last iterate, info says which  */
  SMG_EHIP = -3,        /* a HIP runtime call failed                       */
  SMG_EWORKSPACE = -4,  /* workspace missing, too small or misaligned      */
  SMG_ESTATE = -5       /* call out of order (e.g. solve before setup)     */
} smg_status;

enum { SMG_SPHERICAL = 0, SMG_CYLINDRICAL = 1 };
enum { SMG_RADIAL_UNIFORM = 0, SMG_RADIAL_LOG = 1 };
enum { SMG_FP64 = 0, SMG_MIXED = 1 };
enum { SMG_DGF_AUTO = 0, SMG_DGF_AUX = 1, SMG_DGF_EXTENDED = 2 };
enum { SMG_LINE_SOR = 0, SMG_LINE_EXACT = 1 };
/* nu_pre = nu_post = SMG_NU_AUTO: smoothing steps chosen by the library at
 * setup: 1 each way when every problem's finest level is too large for the
 * fused in-LDS V-cycle (each step there costs two whole-grid launches), 2 when
 * the whole V-cycle runs in that kernel. */
enum { SMG_NU_AUTO = -1 };

/* Grid of Sec. 2.1.  Radial faces: uniform, or geometric
 * a_min * (a_max/a_min)^(f/n_a) for SMG_RADIAL_LOG.  b faces are uniform;
 * b_min = 0 (and b_max = pi) are poles for spherical grids.
 * Constraints (SMG_EINVAL otherwise): n_a, n_b >= 4 and even; n_phi even,
 * >= 4, of the form 2^p 3^q with n_phi/2 <= 1024; 0 < a_min < a_max;
 * spherical b range within [0, pi]; the inner radial ghost face
 * a_min - (a_max - a_min)/n_a > 0 for uniform grids; G > 0. */
typedef struct {
  int geometry;          /* SMG_SPHERICAL | SMG_CYLINDRICAL */
  int radial;            /* SMG_RADIAL_UNIFORM | SMG_RADIAL_LOG */
  int n_a, n_b, n_phi;
  double a_min, a_max;
  double b_min, b_max;
  double G;
} smg_grid;

/* Solver options.  Zero-initialised fields take the defaults in brackets. */
typedef struct {
  int precision;         /* SMG_FP64 [default] | SMG_MIXED (FP32 smoothing
                            and transfers, FP64 residual, coarsest solve and
                            correction accumulation: iterative refinement) */
  int nu_pre;            /* pre-smoothing steps per level [2]; SMG_NU_AUTO */
  int nu_post;           /* post-smoothing steps per level [2]; SMG_NU_AUTO */
  int n_sor;             /* SOR passes per line relaxation [2] (Sec. 3.2) */
  int max_cycles;        /* V-cycles per mode and solve [60] */
  int dgf_method;        /* SMG_DGF_AUTO [log radial -> extended domain,
                            uniform -> auxiliary grid] | _AUX | _EXTENDED */
  int n_pad;             /* DGF padding cells [16] (Sec. 4.2) */
  double dgf_tol;        /* relative residual of the DGF solves [1e-13] */
  int line_solver;       /* SMG_LINE_SOR [default]: each line relaxed by
                            n_sor even-odd SOR passes with the WKB omega
                            (Sec. 3.2); SMG_LINE_EXACT: each line solved
                            exactly (Thomas), the ideal Sec. 3.2 names.  The
                            DGF extended-domain solves always use exact
                            lines (their radial cells reach aspect ratios
                            of 1e3 and more). */
  int launch;            /* SMG_LAUNCH_GRAPH [default]: after the first solve
                            of a kind (zero guess; warm start, told apart by
                            the number of solutions its extrapolation uses
                            and by the learned guess) every V-cycle of a
                            solve is scheduled from the previous solve's
                            per-mode cycle counts, the whole body (both
                            multigrid solves and the boundary steps) replays
                            as one captured HIP graph, and the host
                            synchronises once per solve; modes that still
                            miss the tolerance are finished afterwards.
                            SMG_LAUNCH_DYNAMIC: the host reads the number of
                            unconverged modes after every V-cycle (no graph). */
  int autotune;          /* 1: at setup, time V-cycles under candidate launch
                            shapes (where the in-LDS coarse cycle starts,
                            smoother blocks per launch) for the plane-count
                            buckets up to 2, 8, 32 and all planes, each at
                            its top, middle and bottom count, and keep the
                            fastest [0: built-in rule] */
  int coarse_cells;      /* coarsening stops at the first level with at most
                            this many cells, after at least one halving (the
                            paper leaves the depth open, Sec. 3.3); that level
                            is solved exactly by fast diagonalisation
                            [0: 128] */
  int coarse_solver;     /* SMG_COARSE_EXACT [default]: the coarsest level
                            solved exactly by fast diagonalisation (falls
                            back to red-black SOR where the factors fail
                            their check); SMG_COARSE_SOR: red-black point
                            SOR with the 2D omega of Appendix A, from zero
                            until the residual drops by 1e-10 (Sec. 3.3; the
                            coarsest level must then have <= 1024 cells) */
  int warm_extrapolate;  /* order of the extrapolated warm start (flag
                            SMG_WARM_EXTRAP), 0 to 3: the plan keeps that
                            many solutions before the last one and warm
                            solves start from the polynomial through them
                            (1: 2 u_{t-1} - u_{t-2}; 2: 3 u_{t-1} -
                            3 u_{t-2} + u_{t-3}; 3: 4 u_{t-1} - 6 u_{t-2} +
                            4 u_{t-3} - u_{t-4}); each order costs two more
                            sets of FP64 mode planes of workspace (one per
                            multigrid solve) [0: none] */
} smg_opts;

enum { SMG_COARSE_EXACT = 0, SMG_COARSE_SOR = 1 };

enum { SMG_LAUNCH_GRAPH = 0, SMG_LAUNCH_DYNAMIC = 1 };

/* Per-solve report.  Arrays are caller-owned host buffers of length
 * n_modes = n_phi/2 + 1 (any may be NULL). */
typedef struct {
  int n_modes;
  int *cycles1, *cycles2;        /* V-cycles of solve 1 (Psi) and 2 (Phi)   */
  double *resid1, *resid2;       /* final ||D^m||_V / max(||D^m_0||, floor) */
  int total_cycles;              /* sum over modes and both solves          */
  int converged;                 /* 1 if every mode met the tolerance       */
  double ms_fft, ms_mg1, ms_james, ms_mg2, ms_ifft;  /* component times (ms),
                                    measured with HIP events on the stream  */
} smg_info;

/* Flags of smg_solve. */
#define SMG_WARM_PREV   1u  /* start both solves from the previous call's
                               Psi^m / Phi^m (Sec. 5.1, last paragraph);
                               otherwise from zero                         */
#define SMG_TIMINGS     2u  /* fill the component times of smg_info        */
#define SMG_NET_GUESS   4u  /* with SMG_WARM_PREV and an attached network:
                               in the potential's multigrid solve (solve 2,
                               Phi^m) modes 0..m_max start from the
                               network's prediction wherever, after one
                               smoothing step of each, its defect norm is
                               below that of the start they would take
                               otherwise (the extrapolated warm start with
                               SMG_WARM_EXTRAP, else the linear
                               extrapolation of the last two solutions, or
                               the previous solution before two exist);
                               solve 1 (Psi^m) starts them like the other
                               modes.  The multigrid runs to the same
                               tolerance either way.                       */
#define SMG_WARM_EXTRAP 8u  /* with SMG_WARM_PREV on a plan created with
                               opts.warm_extrapolate: each multigrid solve
                               starts its modes from the polynomial
                               extrapolation of its last solutions, of the
                               plan's order or lower while fewer exist
                               (with SMG_NET_GUESS the network's candidate
                               then competes with this start for modes
                               0..m_max); a solve without this flag
                               leaves one usable solution, from which the
                               next starts as u_{t-1}.  Only the
                               cycle count depends on the guess.  SMG_EINVAL
                               on a plan without opts.warm_extrapolate.    */

typedef struct smg_plan smg_plan;

/* Validate the grid and options and build the host tables (geometry,
 * per-level stencil factors, WKB omegas of Appendix A, transfer weights).
 * *out receives a new plan on success.  No device work.
 * Besides the field ranges, the grid must coarsen (halving both sides while
 * both are even, the smaller side stays >= 2 and the coarse inner radial
 * ghost face stays at r > 0) to a level of at most max(128, coarse_cells)
 * cells, or to one whose exact solver exists: n_a = c_a 2^k and n_b =
 * c_b 2^k with small odd c_a, c_b.  SMG_EINVAL otherwise, with the reason
 * the coarsening stopped in smg_last_error (e.g. 130 x 66 stops at the odd
 * 65 x 33). */
smg_status smg_plan_create(const smg_grid *grid, const smg_opts *opts, smg_plan **out);

/* Bytes of device workspace the plan needs (DGF tables, mode planes of every
 * multigrid level, previous-step solutions, tables).  0 on a NULL plan. */
size_t smg_workspace_bytes(const smg_plan *plan);

/* Bind the caller's workspace (>= smg_workspace_bytes, 256-byte aligned),
 * upload the tables and compute the discrete Green's function tables of
 * Sec. 4.2 on the device (one-time, not part of a solve).  Temporary device
 * memory of the DGF computation is allocated and freed inside this call;
 * with opts.autotune the launch shapes are tuned here.  The plan owns the
 * HIP graphs of later solves and a private stream they are captured on. */
smg_status smg_plan_setup(smg_plan *plan, void *workspace_dev, size_t workspace_bytes, void *stream);

/* The seven-step workflow of Sec. 5.1: rho_dev -> phi_dev, both
 * [n_a][n_b][n_phi] FP64 device arrays (may not alias).  Each mode iterates
 * until ||D^m||_V <= rel_tol * max(||D^m_0||_V, 1e-6 max_m ||D^m_0||_V)
 * (D_0: defect of the zero guess with the solve's boundary data).
 * info_host may be NULL.  Returns SMG_ENOCONV if a mode hits max_cycles. */
smg_status smg_solve(smg_plan *plan, const double *rho_dev, double *phi_dev, double rel_tol,
                     unsigned flags, void *stream, smg_info *info_host);

/* Destroy a plan (the workspace stays the caller's).  NULL is a no-op. */
smg_status smg_plan_destroy(smg_plan *plan);

/* Thread-local message of the last failing call ("" if none). */
const char *smg_last_error(void);

/* ---- batches: several problems in every launch ---------------------------
 * The multigrid solves of several set-up plans run together: every kernel
 * launch of a V-cycle covers the unconverged mode planes of all plans (each
 * with its own grid, tables and launch shape), the convergence lists span
 * the batch, and the per-mode cycle schedule and graph replay of the
 * SMG_LAUNCH_GRAPH form apply to the batch as a whole.  The plans must share
 * precision, line solver, nu_pre, nu_post and n_sor (SMG_EINVAL), hold at
 * most 4096 mode planes together, and stay set up while the batch is used.
 * Each plan keeps its own workspace (its mode arrays are the ones solved);
 * the batch needs a small workspace of its own for its tables and lists.
 * A batch solve and a solve of one of its plans must not overlap in time;
 * SMG_WARM_PREV starts from the plans' last Psi^m / Phi^m. */
typedef struct smg_batch smg_batch;
smg_status smg_batch_create(smg_plan *const *plans, int n_plans, smg_batch **out);
size_t smg_batch_workspace_bytes(const smg_batch *batch);
/* Bind the batch workspace (256-byte aligned); tunes the launch shapes of
 * the batch when plans[0] was created with opts.autotune. */
smg_status smg_batch_setup(smg_batch *batch, void *workspace_dev, size_t workspace_bytes, void *stream);
/* rho_dev[q] -> phi_dev[q] for plan q as smg_solve does; infos_host: NULL or
 * n_plans reports (component times are those of the whole batch). */
smg_status smg_batch_solve(smg_batch *batch, const double *const *rho_dev, double *const *phi_dev, double rel_tol,
                           unsigned flags, void *stream, smg_info *infos_host);
const char *smg_batch_tune_report(const smg_batch *batch);
smg_status smg_batch_destroy(smg_batch *batch);

/* ---- the learned initial guess --------------------------------------------
 * A U-Net on real mode planes (one image per real or imaginary part of a
 * low-m mode), 8 input channels (f_t / s_f, (f_t - f_{t-1}) / s_d,
 * u_{t-1} / s_u, m / 4, (i + 1/2) / n_a - 1/2, (j + 1/2) / n_b - 1/2,
 * and this part of (u_{t-1} - u_{t-2}) / s_o and of -i (u_{t-1} - u_{t-2})
 * / s_o (the other part, signed as a small rotation of the mode changes
 * it); s_f, s_d, s_u the plane RMS of f_t,
 * f_t - f_{t-1} and u_{t-1}, s_o the RMS of u_{t-1} - u_{t-2}) and one
 * output channel, the correction (u_t - 2 u_{t-1} + u_{t-2}) / s_o to the
 * linear extrapolation of the last two solutions.  At each
 * of `levels` resolutions two 3x3 convolutions with ReLU (32 channels),
 * 2x2 average pooling down, nearest upsampling and concatenation with the
 * encoder output up, a 1x1 output layer.  Weights and activations are BF16,
 * products accumulate in FP32 on the matrix cores; the master parameters,
 * their gradients and the Adam moments are FP32.
 *
 * Parameter vector (FP32, n = smg_net_param_count): per layer in the order
 * encoder levels 0..levels-1 (two 3x3 layers each), decoder levels
 * levels-2..0 (two 3x3 layers each, the first reading 64 channels), the
 * 1x1 output layer; per layer the weights [c_out][9][c_in] (tap 3(dy+1) +
 * (dx+1) reads pixel (y+dy, x+dx)) or [c_out][c_in], then the biases.
 * Images are NHWC FP32 arrays [n][h][w][8] in, [n][h][w] out; h and w are
 * multiples of 2^(levels-1).  The caller owns all device memory: the
 * state buffer (parameters, gradients, Adam moments, BF16 copy) and the
 * work buffer of one batch shape (activations and their gradients). */
typedef struct smg_net smg_net;
smg_status smg_net_create(int levels, int channels /* 32 */, smg_net **out);
smg_status smg_net_destroy(smg_net *net);
long long smg_net_param_count(const smg_net *net);
size_t smg_net_state_bytes(const smg_net *net);
/* Bind the state buffer (256-byte aligned); parameters start at zero. */
smg_status smg_net_bind(smg_net *net, void *state_dev, size_t state_bytes, void *stream);
/* Copy FP32 parameters in (device array; Adam moments reset) or out. */
smg_status smg_net_set_params(smg_net *net, const float *params_dev, void *stream);
smg_status smg_net_get_params(const smg_net *net, float *params_dev, void *stream);
/* Gradients of the last smg_net_backward / smg_net_train_step. */
smg_status smg_net_get_grads(const smg_net *net, float *grads_dev, void *stream);
/* Bytes of the work buffer for n images of h x w (0 if the shape is invalid). */
size_t smg_net_work_bytes(const smg_net *net, int n, int h, int w);
/* y = net(x); y_dev may be NULL (the output stays in the work buffer). */
smg_status smg_net_forward(smg_net *net, const float *x_dev, float *y_dev, int n, int h, int w, void *work_dev,
                           size_t work_bytes, void *stream);
/* After smg_net_forward on the same work buffer: gradients of
 * sum(dy * y) with respect to the parameters (readable with
 * smg_net_get_grads). */
smg_status smg_net_backward(smg_net *net, const float *dy_dev, int n, int h, int w, void *work_dev, size_t work_bytes,
                            void *stream);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8) on the mean squared error of
 * n samples picked by idx_host (each in [0, n_samples)) from samples_dev
 * (each sample: x [h][w][8] then the target [h][w], FP32).  loss_host (may
 * be NULL) receives the batch loss before the step (synchronises). */
smg_status smg_net_train_step(smg_net *net, const float *samples_dev, int n_samples, const int *idx_host, int n, int h,
                              int w, float lr, void *work_dev, size_t work_bytes, void *stream, float *loss_host);

/* ---- single layers of the network, for layer-level checks ----------------
 * BF16 arrays are uint16 bit patterns (round to nearest even).  Images are
 * NHWC: x[n][h][w][c_in], zero outside the image.
 *
 * smg_net_conv3: one 3x3 'same' convolution (a layer of the learned-guess
 * U-Net): y[q][i][j][o] = bf16(act(b[o] + sum_{t,c} W[o][t][c] x[q][i+dy_t][j+dx_t][c]))
 * with tap t = 3 (dy + 1) + (dx + 1), act = ReLU when relu != 0, b may be
 * NULL (zero bias); sums in FP32.  W is BF16 [c_out][9][c_in], b FP32
 * [c_out], y BF16 [n][h][w][c_out].  c_in a multiple of 8 in [8, 64],
 * c_out = 32 (SMG_EINVAL otherwise).  Enqueued on `stream`.
 *
 * smg_net_conv3_wgrad: the parameter gradients of that layer for an output
 * gradient g[n][h][w][c_out] (BF16): dW[o][t][c] = sum_pixels g[p][o]
 * x[p + tap t][c], db[o] = sum_pixels g[p][o], both FP32 and overwritten.
 * work_dev is scratch of smg_net_conv3_wgrad_work_bytes bytes (per-chunk
 * partial sums; SMG_EWORKSPACE if smaller). */
smg_status smg_net_conv3(const unsigned short *x_dev, int c_in, const unsigned short *w_dev, const float *b_dev,
                         unsigned short *y_dev, int c_out, int relu, int n, int h, int w, void *stream);
size_t smg_net_conv3_wgrad_work_bytes(int c_in, int c_out, int n, int h, int w);
smg_status smg_net_conv3_wgrad(const unsigned short *g_dev, int c_out, const unsigned short *x_dev, int c_in,
                               float *dw_dev, float *db_dev, int n, int h, int w, void *work_dev, size_t work_bytes,
                               void *stream);
/* smg_net_conv3_wgrad for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and results (dW bit for bit; db up to the
 * order of its FP32 atomic additions), with the per-chunk partial sums in
 * a static 8 MiB device array instead of a work buffer.  Calls no
 * allocating routine.  Each GPU holds its own array from the first call on
 * it until the process ends; every call on that GPU shares it, so calls
 * that overlap on one GPU (other streams, other threads) race and must be
 * serialised by the caller.  SMG_EINVAL beyond n*h*w = 2^28 pixels (the
 * pixel chunks grow so that the partial sums of any layer fit the array). */
smg_status smg_net_conv3_wgrad_noalloc(const unsigned short *g_dev, int c_out, const unsigned short *x_dev, int c_in,
                                       float *dw_dev, float *db_dev, int n, int h, int w, void *stream);

/* ---- the learned guess in a plan's solves ---------------------------------
 * Attach a bound network as the initial-guess model of modes 0..m_max
 * (m_max <= 8; n_a and n_b divisible by 2^(levels-1)) using a caller-owned
 * work buffer of smg_plan_net_work_bytes bytes (256-byte aligned).  From
 * then on every solve keeps the potential's right-hand side of those modes
 * for the next step (that of solve 1 too while samples are recorded); a
 * warm-started solve with SMG_NET_GUESS builds the network inputs
 * (per real image: f_t / s_f, (f_t - f_{t-1}) / s_d, u_{t-1} / s_u, m / 4,
 * the two normalised grid coordinates, this part of (u_{t-1} - u_{t-2}) /
 * s_o and of -i (u_{t-1} - u_{t-2}) / s_o, with s_f, s_d, s_u the plane RMS
 * values of f_t, f_t - f_{t-1} and u_{t-1}, and s_o, the scale of the
 * output, the RMS of u_{t-1} - u_{t-2}; before two warm steps have run,
 * and for a static plane (last change below 1e-4 of its RMS), channels 6
 * and 7 are zero) before the potential's multigrid solve (solve 2) and
 * starts every mode from the better (defect norms after one smoothing step
 * of each) of the candidate, the baseline u_{t-1} + (u_{t-1} - u_{t-2}) (the
 * linear extrapolation; u_{t-1} before u_{t-2} exists, and on a static
 * part) plus s_o y, the network's correction y, and the start the mode
 * would take otherwise: the plan's extrapolated warm start where
 * SMG_WARM_EXTRAP applies one, else that baseline.  While samples are
 * recorded (smg_plan_record), the inputs are built for both solves (as
 * training samples; without SMG_NET_GUESS too), but the modes of solve 1
 * take no network guess; otherwise a solve builds inputs only for the
 * network's guess.
 * A NULL net detaches. */
size_t smg_plan_net_work_bytes(const smg_plan *plan, const smg_net *net, int m_max);
smg_status smg_plan_attach_net(smg_plan *plan, smg_net *net, int m_max, void *work_dev, size_t work_bytes,
                               void *stream);
/* Record training samples: every later warm-started solve that has the
 * solutions of the two previous steps (from the third solve of a sequence
 * on; for solve 1, counted from the first solve recorded) appends, for each of its two multigrid solves and each real image of
 * modes 0..m_max, the sample (network input [n_a][n_b][8], target
 * (u_t - 2 u_{t-1} + u_{t-2}) / s_o [n_a][n_b] -- the correction to the
 * linear extrapolation, FP32) to samples_dev while fewer than `capacity` are stored
 * (the layout smg_net_train_step reads).  Resets the count; capacity 0 stops
 * recording.  smg_plan_recorded returns the count (synchronises). */
smg_status smg_plan_record(smg_plan *plan, float *samples_dev, int capacity, void *stream);
int smg_plan_recorded(const smg_plan *plan, void *stream);
/* Which modes took the network's guess in the last SMG_NET_GUESS solve:
 * used_host[t * (m_max + 1) + m] for solve t = 0 (Psi: always 0), 1 (Phi). */
smg_status smg_plan_net_used(const smg_plan *plan, int *used_host, void *stream);
/* The learned-guess step of multigrid solve t (0: Psi, 1: Phi) of a
 * warm-started SMG_NET_GUESS solve, on caller planes, for step-level checks.
 * Inputs, complex FP64 [m_max+1][n_a][n_b] (modes 0..m_max): f_dev this
 * step's right-hand side of solve t (for t = 1 with the ghost potential
 * folded in), fprev_dev the previous step's, uprev_dev the previous step's
 * solution, uprev2_dev (may be NULL) the solution of the step before.
 * Outputs: guess_dev (same layout) the initial guess each mode
 * starts from (the network's candidate u_prev + s_o y or u_prev, by the
 * defect norms after one smoothing step of each); x_dev (may be NULL) the
 * FP32 network inputs [2 m_max + 1][n_a][n_b][8] (image 0 = Re m=0, 2m-1 =
 * Re m, 2m = Im m); y_dev (may be NULL) the FP32 network outputs
 * [2 m_max + 1][n_a][n_b]; used_host (may be NULL) int [m_max+1], 1 where
 * the network's candidate was taken.  Synchronises.  Overwrites the plan's
 * solve state, so the next smg_solve starts cold.  SMG_ESTATE without an
 * attached network. */
smg_status smg_net_guess_step(smg_plan *plan, int t, const double *f_dev, const double *fprev_dev,
                              const double *uprev_dev, const double *uprev2_dev, double *guess_dev, float *x_dev,
                              float *y_dev, int *used_host, void *stream);

/* ---- geometry query (host, no device work) ------------------------------ */
/* Cell-centre coordinates: a_host[n_a], b_host[n_b], phi_host[n_phi]
 * (volume-weighted centroids of Eq. cell_centers_sph and Sec. 2.1.2), and
 * the cell volumes dv_host[n_a*n_b] (per azimuthal cell, Eqs. vol_sph /
 * vol_cyl).  Any pointer may be NULL. */
smg_status smg_plan_geometry(const smg_plan *plan, double *a_host, double *b_host, double *phi_host,
                             double *dv_host);

/* Number of multigrid levels, number of boundary ghost cells n_g of the
 * James boundary, and the level sizes (n_a, n_b per level; arrays of 16). */
smg_status smg_plan_shape(const smg_plan *plan, int *n_levels, int *n_ghost, int *level_na, int *level_nb);

/* ---- the steps of the path, for step-level checks ------------------------
 * Each runs one step of smg_solve on caller buffers; all arrays are device
 * arrays in the layouts above.  The plan must be set up. */

/* Step 2 (Sec. 2.2): modes_dev[m] = 4 pi G / n_phi * sum_k rho_k e^{-2 pi i m k/n_phi}. */
smg_status smg_fft_forward(smg_plan *plan, const double *rho_dev, double *modes_dev, void *stream);

/* Step 7: phi_k = sum_{m=0}^{n_phi-1} X_m e^{+2 pi i m k/n_phi} with the upper
 * half completed by Hermitian symmetry (imaginary parts of m = 0 and
 * m = n_phi/2 ignored). */
smg_status smg_fft_inverse(smg_plan *plan, const double *modes_dev, double *phi_dev, void *stream);

/* Steps 3/6 for given right-hand sides: solve L_m u^m = f^m for every mode
 * with homogeneous boundary conditions (the boundary data of solve 2 are
 * already folded into f).  u_dev holds the initial guess on entry and the
 * solution on exit.  cycles_host / resid_host (length n_modes) may be NULL. */
smg_status smg_mg_solve(smg_plan *plan, const double *f_dev, double *u_dev, double rel_tol,
                        void *stream, int *cycles_host, double *resid_host);

/* One V-cycle on every mode (no convergence test).  This and the next two
 * entry points need an FP64 plan (SMG_EINVAL otherwise).  The step entry
 * points work on copies in the plan's own arrays, so the next smg_solve does
 * not warm-start. */
smg_status smg_mg_vcycle(smg_plan *plan, const double *f_dev, double *u_dev, void *stream);

/* One smoothing step (radial-line phase then polar-line phase, Algorithm 1)
 * on the finest level for every mode. */
smg_status smg_mg_smooth(smg_plan *plan, const double *f_dev, double *u_dev, void *stream);

/* Residual f - L_m u (finest level, every mode) into r_dev. */
smg_status smg_mg_residual(smg_plan *plan, const double *f_dev, const double *u_dev, double *r_dev,
                           void *stream);

/* Steps 4-5 (Eqs. charge_sph / charge_cyl and theta_left..theta_top):
 * sigma_dev[m][g] = screening masses from psi_dev; theta_dev[m][g] =
 * sum_s Gt^m(g <- s) sigma^m_s; f2_dev = f_dev with the ghost potential
 * -Theta folded into the boundary cells.  sigma/theta are complex
 * [n_modes][n_g]. */
smg_status smg_james(smg_plan *plan, const double *psi_dev, const double *f_dev, double *sigma_dev,
                     double *theta_dev, double *f2_dev, void *stream);

/* Gravitational acceleration g = -grad Phi on every cell face (Sec. 2.1,
 * Eq. gradient): the potential difference of the two cells sharing a face
 * over the distance of their centroids projected on the face normal --
 * radial faces a_{i+1} - a_i; theta faces r_i (theta_{j+1} - theta_j) or z
 * faces z_{j+1} - z_j; azimuthal faces r_i sin(theta_j) dphi (spherical) or
 * R_i dphi (cylindrical).  Boundary faces use the ghost potential -Theta of
 * the second solve (Sec. 4) transformed back to phi; faces lying on a pole
 * carry 0.
 *   phi_dev    [n_r][n_b][n_phi] FP64 potential (as returned by smg_solve)
 *   theta_dev  complex [n_modes][n_g] screening potential Theta^m (as from
 *              smg_james), or NULL for the Theta of the plan's most recent
 *              solve, alone or in a batch (SMG_ESTATE if there is none);
 *              that Theta is read when the work runs, so enqueue this on the
 *              solve's stream or after it has finished
 *   g_a_dev    [n_r + 1][n_b][n_phi] radial faces (index i: face i - 1/2)
 *   g_b_dev    [n_r][n_b + 1][n_phi] theta / z faces (index j: face j - 1/2)
 *   g_phi_dev  [n_r][n_b][n_phi] azimuthal faces (index k: face k + 1/2,
 *              periodic)
 * Components point along the increasing coordinate.  All device buffers are
 * caller-owned; the work is enqueued on `stream` (uses the plan's ghost
 * scratch, so calls on one plan must not overlap). */
smg_status smg_acceleration(smg_plan *plan, const double *phi_dev, const double *theta_dev, double *g_a_dev,
                            double *g_b_dev, double *g_phi_dev, void *stream);

/* Copy the DGF table Gt^m(t <- s) of mode m to dgf_host[n_g][n_g] (FP64,
 * row = field ghost t, column = source ghost s). */
smg_status smg_dgf_table(smg_plan *plan, int m, double *dgf_host, void *stream);

/* ---- per-launch timing ---------------------------------------------------
 * Between smg_profile_begin and smg_profile_end every kernel launch of
 * smg_solve is bracketed by HIP events on the solve's stream.  Once an
 * earlier solve of the plan gave the per-mode cycle schedule, a profiled
 * solve enqueues the scheduled launches from the host (the launches a graph
 * replay makes, without the graph), so the durations are those of the
 * replayed launches; before that it runs the per-cycle host loop.  End
 * synchronises the device and reports, per kernel class, the number of
 * launches, the summed launch durations (ms) and the summed algorithmic
 * bytes (each launch reads its inputs and writes its outputs once: 48 B per
 * cell for a directional FP64 smoothing pass, 40 B per fine cell for the
 * fused residual + restriction, 36 B for prolongation + correction, the
 * real input plus complex output for the FFTs, the FP64 DGF table for the
 * boundary convolution).  `name` points to a string owned by the library.
 * Writes at most max_stats entries; *n_stats receives the number of classes. */
typedef struct {
  const char *name;
  int launches;
  double total_ms;
  double bytes;
} smg_kernel_stat;

smg_status smg_profile_begin(smg_plan *plan);
smg_status smg_profile_end(smg_plan *plan, smg_kernel_stat *stats, int max_stats, int *n_stats);

/* Text report of the setup-time autotuner (opts.autotune = 1): the timed
 * candidates and the configuration kept per planes bucket.  Owned by the
 * plan; empty when the autotuner did not run. */
const char *smg_tune_report(const smg_plan *plan);

#ifdef __cplusplus
}
#endif
#endif /* SMG_H */
