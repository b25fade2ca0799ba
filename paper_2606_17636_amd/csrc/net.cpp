// Host side of the learned initial guess (include/smg.h, smg_net_*): the
// U-Net's parameter layout, its activation workspace, forward and backward
// passes as sequences of the kernels in net.hip, MSE training steps with
// Adam.
#include <hip/hip_runtime.h>

#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "net_internal.h"
#include "netdef.h"
#include "smg.h"
#include "smg_internal.h"

using namespace smg;

namespace smg {
void set_error(const std::string& msg);
}

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

smg_status nfail(smg_status s, const std::string& m) {
  set_error(m);
  return s;
}

#define NCHK(expr)                                                                          \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return nfail(SMG_EHIP, strprintf("%s failed: %s", #expr, hipGetErrorString(e_))); \
  } while (0)
#define NST(expr)                \
  do {                           \
    smg_status s_ = (expr);      \
    if (s_ != SMG_OK) return s_; \
  } while (0)

}  // namespace

// ---------------------------------------------------------------------------
// workspace of one batch shape
// ---------------------------------------------------------------------------
NetWork NetDef::work_layout(int n, int H, int W) const {
  NetWork w{};
  w.n = n; w.H = H; w.W = W;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
  const size_t bf = sizeof(unsigned short);
  const size_t np0 = (size_t)n * H * W;
  w.x32 = take(sizeof(float) * np0 * in_ch);
  w.xb = take(bf * np0 * in_ch);
  w.y = take(sizeof(float) * np0);
  w.gy = take(sizeof(float) * np0);
  w.tgt = take(sizeof(float) * np0);
  for (int l = 0; l < levels; ++l) {
    const size_t np = (size_t)n * (H >> l) * (W >> l);
    w.h[l] = l > 0 ? take(bf * np * ch) : 0;
    w.a[l] = take(bf * np * ch);
    w.cat[l] = l < levels - 1 ? take(bf * np * 2 * ch) : 0;
    w.ebot = l == levels - 1 ? take(bf * np * ch) : w.ebot;
    w.ad[l] = l < levels - 1 ? take(bf * np * ch) : 0;
    w.d[l] = l < levels - 1 ? take(bf * np * ch) : 0;
    w.g32a[l] = take(bf * np * ch);
    w.g32b[l] = take(bf * np * ch);
    w.g64[l] = l < levels - 1 ? take(bf * np * 2 * ch) : 0;
  }
  // the largest layer's weight-gradient partials (the 2 ch -> ch decoder input layer)
  w.part_floats = std::max(smgn::wgrad_partials((int)np0, ch, 2 * ch), smgn::wgrad_partials((int)np0, ch, in_ch));
  w.part = take(sizeof(float) * w.part_floats);
  w.bytes = off;
  return w;
}

NetDef::NetDef(int levels_, int ch_, int in_ch_) : levels(levels_), ch(ch_), in_ch(in_ch_) {
  int cin = in_ch;
  size_t off = 0;
  auto add = [&](int kind, int ci, int co) {
    NetLayer L{kind, ci, co, off, 0};
    off += (size_t)co * ci * (kind == 3 ? 9 : 1);
    L.b_off = off;
    off += co;
    layers.push_back(L);
  };
  for (int l = 0; l < levels; ++l) {
    add(3, cin, ch);
    add(3, ch, ch);
    cin = ch;
  }
  for (int l = 0; l < levels - 1; ++l) {
    add(3, 2 * ch, ch);
    add(3, ch, ch);
  }
  add(1, ch, 1);
  n_params = off;
}

size_t NetDef::state_bytes() const {
  const size_t np = n_params;
  return align_up(sizeof(float) * np) * 4 + align_up(sizeof(unsigned short) * np) +
         align_up(sizeof(unsigned short) * 9 * 2 * ch * ch) + align_up(sizeof(float) * 4);
}

void NetDef::bind(char* s) {
  const size_t np = n_params;
  size_t off = 0;
  auto take = [&](size_t bytes) { char* r = s + off; off = align_up(off + bytes); return r; };
  p = reinterpret_cast<float*>(take(sizeof(float) * np));
  g = reinterpret_cast<float*>(take(sizeof(float) * np));
  m = reinterpret_cast<float*>(take(sizeof(float) * np));
  v = reinterpret_cast<float*>(take(sizeof(float) * np));
  pb = reinterpret_cast<unsigned short*>(take(sizeof(unsigned short) * np));
  wflip = reinterpret_cast<unsigned short*>(take(sizeof(unsigned short) * 9 * 2 * ch * ch));
  loss = reinterpret_cast<float*>(take(sizeof(float) * 4));
}

// ---------------------------------------------------------------------------
// forward / backward
// ---------------------------------------------------------------------------
smg_status NetDef::forward(char* base, const NetWork& w, hipStream_t st, bool train) const {
  auto B = [&](size_t off) { return reinterpret_cast<unsigned short*>(base + off); };
  const int n = w.n;
  const size_t np0 = (size_t)n * w.H * w.W;
  NCHK(smgn::to_bf16(reinterpret_cast<const float*>(base + w.x32), B(w.xb), np0 * in_ch, st));
  const NetLayer& LO = layers.back();
  float* y = reinterpret_cast<float*>(base + w.y);
  int k = 0;
  for (int l = 0; l < levels; ++l) {
    const int H = w.H >> l, W = w.W >> l;
    // level l > 0 reads the pooled copy its level above wrote with its output
    const unsigned short* in = l == 0 ? B(w.xb) : B(w.h[l]);
    const int ics = l == 0 ? in_ch : ch, cin = l == 0 ? in_ch : ch;
    const NetLayer& L0 = layers[k];
    NCHK(smgn::conv3(in, ics, cin, pb + L0.w_off, p + L0.b_off, B(w.a[l]), ch, ch, nullptr, 0, true, n, H, W, st));
    const NetLayer& L1 = layers[k + 1];
    const bool last = l == levels - 1;
    smgn::ConvIn I{B(w.a[l]), nullptr, ch, ch, pb + L1.w_off, p + L1.b_off};
    smgn::ConvOut O{last ? B(w.ebot) : B(w.cat[l]) + ch, last ? ch : 2 * ch, ch, nullptr, 0, true,
                    last ? nullptr : B(w.h[l + 1]), ch, nullptr, nullptr, nullptr};
    if (levels == 1) { O.w1 = pb + LO.w_off; O.b1 = p + LO.b_off; O.y1 = y; }
    NCHK(smgn::conv3x(I, O, n, H, W, st));
    k += 2;
  }
  const unsigned short* dprev = B(w.ebot);
  for (int l = levels - 2; l >= 0; --l) {
    const int H = w.H >> l, W = w.W >> l;
    // the concatenation [upsampled level below, encoder output]: materialised
    // for training (the weight gradient reads it), read in place otherwise
    if (train) NCHK(smgn::up(dprev, ch, B(w.cat[l]), 2 * ch, ch, n, H / 2, W / 2, st));
    const NetLayer& LA = layers[k];
    smgn::ConvIn IA{B(w.cat[l]), train ? nullptr : dprev, 2 * ch, 2 * ch, pb + LA.w_off, p + LA.b_off};
    smgn::ConvOut OA{B(w.ad[l]), ch, ch, nullptr, 0, true, nullptr, 0, nullptr, nullptr, nullptr};
    NCHK(smgn::conv3x(IA, OA, n, H, W, st));
    const NetLayer& LB = layers[k + 1];
    smgn::ConvIn IB{B(w.ad[l]), nullptr, ch, ch, pb + LB.w_off, p + LB.b_off};
    // the top level also computes the 1x1 output layer; its own output is
    // only needed by the backward pass
    smgn::ConvOut OB{(train || l > 0) ? B(w.d[l]) : nullptr, ch, ch, nullptr, 0, true, nullptr, 0, nullptr, nullptr,
                     nullptr};
    if (l == 0) { OB.w1 = pb + LO.w_off; OB.b1 = p + LO.b_off; OB.y1 = y; }
    NCHK(smgn::conv3x(IB, OB, n, H, W, st));
    dprev = B(w.d[l]);
    k += 2;
  }
  return SMG_OK;
}

smg_status NetDef::backward(char* base, const NetWork& w, hipStream_t st) const {
  auto B = [&](size_t off) { return reinterpret_cast<unsigned short*>(base + off); };
  float* part = reinterpret_cast<float*>(base + w.part);
  const int n = w.n;
  const size_t np0 = (size_t)n * w.H * w.W;
  NCHK(smgn::fill_f32(g, n_params, 0.f, st));
  int k = (int)layers.size() - 1;
  const NetLayer& LO = layers[k];
  const unsigned short* d0 = levels > 1 ? B(w.d[0]) : B(w.ebot);
  NCHK(smgn::out_layer_back(reinterpret_cast<const float*>(base + w.gy), d0, ch, pb + LO.w_off, B(w.g32b[0]), ch,
                            (int)np0, g + LO.w_off, g + LO.b_off, st));
  --k;
  // decoder, from the output back; gcur: gradient at the pre-activation of
  // the level's output
  unsigned short* gcur = B(w.g32b[0]);
  for (int l = 0; l <= levels - 2; ++l) {
    const int H = w.H >> l, W = w.W >> l;
    const NetLayer& LB = layers[k];
    const NetLayer& LA = layers[k - 1];
    NCHK(smgn::wgrad(gcur, ch, ch, B(w.ad[l]), ch, ch, part, w.part_floats, g + LB.w_off, g + LB.b_off, n, H, W, st));
    NCHK(smgn::flip_weights(pb + LB.w_off, ch, ch, wflip, st));
    NCHK(smgn::conv3(gcur, ch, ch, wflip, nullptr, B(w.g32a[l]), ch, ch, B(w.ad[l]), ch, false, n, H, W, st));
    NCHK(smgn::wgrad(B(w.g32a[l]), ch, ch, B(w.cat[l]), 2 * ch, 2 * ch, part, w.part_floats, g + LA.w_off, g + LA.b_off, n,
                     H, W, st));
    NCHK(smgn::flip_weights(pb + LA.w_off, ch, 2 * ch, wflip, st));
    NCHK(smgn::conv3(B(w.g32a[l]), ch, ch, wflip, nullptr, B(w.g64[l]), 2 * ch, 2 * ch, nullptr, 0, false, n, H, W, st));
    // through the upsampling into the level below's output
    const unsigned short* below = l + 1 == levels - 1 ? B(w.ebot) : B(w.d[l + 1]);
    NCHK(smgn::up_back(B(w.g64[l]), 2 * ch, below, ch, B(w.g32b[l + 1]), ch, ch, n, H / 2, W / 2, st));
    gcur = B(w.g32b[l + 1]);
    k -= 2;
  }
  // encoder, from the bottom up; gcur is the gradient at the bottom output
  for (int l = levels - 1; l >= 0; --l) {
    const int H = w.H >> l, W = w.W >> l;
    const NetLayer& L1 = layers[2 * l + 1];
    const NetLayer& L0 = layers[2 * l];
    NCHK(smgn::wgrad(gcur, ch, ch, B(w.a[l]), ch, ch, part, w.part_floats, g + L1.w_off, g + L1.b_off, n, H, W, st));
    NCHK(smgn::flip_weights(pb + L1.w_off, ch, ch, wflip, st));
    NCHK(smgn::conv3(gcur, ch, ch, wflip, nullptr, B(w.g32a[l]), ch, ch, B(w.a[l]), ch, false, n, H, W, st));
    const unsigned short* in = l == 0 ? B(w.xb) : B(w.h[l]);
    const int ics = l == 0 ? in_ch : ch, cin = l == 0 ? in_ch : ch;
    NCHK(smgn::wgrad(B(w.g32a[l]), ch, ch, in, ics, cin, part, w.part_floats, g + L0.w_off, g + L0.b_off, n, H, W, st));
    if (l == 0) break;
    // gradient of the pooled input, then into the encoder output above it
    NCHK(smgn::flip_weights(pb + L0.w_off, ch, ch, wflip, st));
    NCHK(smgn::conv3(B(w.g32a[l]), ch, ch, wflip, nullptr, B(w.g32b[l]), ch, ch, nullptr, 0, false, n, H, W, st));
    NCHK(smgn::pool_back(B(w.g32b[l]), ch, B(w.g64[l - 1]) + ch, 2 * ch, B(w.cat[l - 1]) + ch, 2 * ch, B(w.g32b[l - 1]),
                         ch, ch, n, 2 * H, 2 * W, st));
    gcur = B(w.g32b[l - 1]);
  }
  return SMG_OK;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
static smg_status need_net(const smg_net* n) {
  if (!n) return nfail(SMG_EINVAL, "NULL net");
  if (!n->state) return nfail(SMG_ESTATE, "net state not bound (call smg_net_bind first)");
  return SMG_OK;
}

static smg_status check_shape(const smg_net* net, int n, int h, int w) {
  const int q = 1 << (net->def.levels - 1);
  if (n < 1 || h < q || w < q || h % q || w % q)
    return nfail(SMG_EINVAL, strprintf("images must be positive multiples of %d in both sizes", q));
  return SMG_OK;
}

extern "C" smg_status smg_net_create(int levels, int channels, smg_net** out) {
  if (!out) return nfail(SMG_EINVAL, "out must not be NULL");
  *out = nullptr;
  if (levels < 1 || levels > kNetMaxLevels) return nfail(SMG_EINVAL, "levels must be in [1, 6]");
  if (channels != 32) return nfail(SMG_EINVAL, "channels must be 32");
  smg_net* n = new (std::nothrow) smg_net(levels, channels, 8);
  if (!n) return nfail(SMG_EINVAL, "out of host memory");
  *out = n;
  return SMG_OK;
}

extern "C" smg_status smg_net_destroy(smg_net* net) {
  delete net;
  return SMG_OK;
}

extern "C" long long smg_net_param_count(const smg_net* net) { return net ? (long long)net->def.n_params : 0; }

extern "C" size_t smg_net_state_bytes(const smg_net* net) { return net ? net->def.state_bytes() : 0; }

extern "C" smg_status smg_net_bind(smg_net* net, void* state, size_t bytes, void* stream) {
  if (!net || !state) return nfail(SMG_EINVAL, "NULL net or state");
  if (bytes < net->def.state_bytes()) return nfail(SMG_EWORKSPACE, "net state buffer too small");
  if (reinterpret_cast<uintptr_t>(state) % kAlign) return nfail(SMG_EWORKSPACE, "net state must be 256-byte aligned");
  net->state = static_cast<char*>(state);
  net->def.bind(net->state);
  net->step = 0;
  hipStream_t st = static_cast<hipStream_t>(stream);
  NCHK(smgn::fill_f32(net->def.p, 4 * align_up(sizeof(float) * net->def.n_params) / sizeof(float), 0.f, st));
  NCHK(smgn::params_bf16(net->def.p, net->def.pb, (int)net->def.n_params, st));
  return SMG_OK;
}

extern "C" smg_status smg_net_set_params(smg_net* net, const float* params, void* stream) {
  NST(need_net(net));
  hipStream_t st = static_cast<hipStream_t>(stream);
  NCHK(hipMemcpyAsync(net->def.p, params, sizeof(float) * net->def.n_params, hipMemcpyDeviceToDevice, st));
  NCHK(smgn::fill_f32(net->def.m, net->def.n_params, 0.f, st));
  NCHK(smgn::fill_f32(net->def.v, net->def.n_params, 0.f, st));
  NCHK(smgn::params_bf16(net->def.p, net->def.pb, (int)net->def.n_params, st));
  net->step = 0;
  return SMG_OK;
}

extern "C" smg_status smg_net_get_params(const smg_net* net, float* params, void* stream) {
  NST(need_net(net));
  NCHK(hipMemcpyAsync(params, net->def.p, sizeof(float) * net->def.n_params, hipMemcpyDeviceToDevice,
                      static_cast<hipStream_t>(stream)));
  return SMG_OK;
}

extern "C" smg_status smg_net_get_grads(const smg_net* net, float* grads, void* stream) {
  NST(need_net(net));
  NCHK(hipMemcpyAsync(grads, net->def.g, sizeof(float) * net->def.n_params, hipMemcpyDeviceToDevice,
                      static_cast<hipStream_t>(stream)));
  return SMG_OK;
}

extern "C" size_t smg_net_work_bytes(const smg_net* net, int n, int h, int w) {
  if (!net || check_shape(net, n, h, w) != SMG_OK) return 0;
  return net->def.work_layout(n, h, w).bytes;
}

static smg_status work_ok(const smg_net* net, int n, int h, int w, void* work, size_t bytes, NetWork* out) {
  NST(need_net(net));
  NST(check_shape(net, n, h, w));
  *out = net->def.work_layout(n, h, w);
  if (!work || bytes < out->bytes) return nfail(SMG_EWORKSPACE, strprintf("net work buffer of %zu bytes needed", out->bytes));
  if (reinterpret_cast<uintptr_t>(work) % kAlign) return nfail(SMG_EWORKSPACE, "net work buffer must be 256-byte aligned");
  return SMG_OK;
}

extern "C" smg_status smg_net_forward(smg_net* net, const float* x, float* y, int n, int h, int w, void* work,
                                      size_t bytes, void* stream) {
  NetWork wl;
  NST(work_ok(net, n, h, w, work, bytes, &wl));
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(work);
  const size_t np0 = (size_t)n * h * w;
  NCHK(hipMemcpyAsync(base + wl.x32, x, sizeof(float) * np0 * net->def.in_ch, hipMemcpyDeviceToDevice, st));
  // the forward the backward pass follows (it keeps every activation)
  NST(net->def.forward(base, wl, st, true));
  if (y) NCHK(hipMemcpyAsync(y, base + wl.y, sizeof(float) * np0, hipMemcpyDeviceToDevice, st));
  return SMG_OK;
}

extern "C" smg_status smg_net_backward(smg_net* net, const float* dy, int n, int h, int w, void* work, size_t bytes,
                                       void* stream) {
  NetWork wl;
  NST(work_ok(net, n, h, w, work, bytes, &wl));
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(work);
  NCHK(hipMemcpyAsync(base + wl.gy, dy, sizeof(float) * (size_t)n * h * w, hipMemcpyDeviceToDevice, st));
  return net->def.backward(base, wl, st);
}

extern "C" smg_status smg_net_train_step(smg_net* net, const float* samples, int n_samples, const int* idx, int n,
                                         int h, int w, float lr, void* work, size_t bytes, void* stream,
                                         float* loss_host) {
  NetWork wl;
  NST(work_ok(net, n, h, w, work, bytes, &wl));
  if (!samples || !idx) return nfail(SMG_EINVAL, "samples and idx must not be NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(work);
  const size_t img = (size_t)h * w, stride = img * (net->def.in_ch + 1);
  for (int q = 0; q < n; ++q) {
    if (idx[q] < 0 || idx[q] >= n_samples) return nfail(SMG_EINVAL, "sample index out of range");
    const float* s = samples + (size_t)idx[q] * stride;
    NCHK(hipMemcpyAsync(base + wl.x32 + sizeof(float) * img * net->def.in_ch * q, s,
                        sizeof(float) * img * net->def.in_ch, hipMemcpyDeviceToDevice, st));
    NCHK(hipMemcpyAsync(base + wl.tgt + sizeof(float) * img * q, s + img * net->def.in_ch, sizeof(float) * img,
                        hipMemcpyDeviceToDevice, st));
  }
  NST(net->def.forward(base, wl, st, true));
  NCHK(smgn::fill_f32(net->def.loss, 1, 0.f, st));
  NCHK(smgn::mse(reinterpret_cast<float*>(base + wl.y), reinterpret_cast<float*>(base + wl.tgt),
                 reinterpret_cast<float*>(base + wl.gy), (int)(img * n), net->def.loss, st));
  NST(net->def.backward(base, wl, st));
  net->step += 1;
  NCHK(smgn::adam(net->def.p, net->def.g, net->def.m, net->def.v, net->def.pb, (int)net->def.n_params, lr, 0.9f, 0.999f,
                  1e-8f, net->step, st));
  if (loss_host) {
    NCHK(hipMemcpyAsync(loss_host, net->def.loss, sizeof(float), hipMemcpyDeviceToHost, st));
    NCHK(hipStreamSynchronize(st));
  }
  return SMG_OK;
}

// ---------------------------------------------------------------------------
// single layers, for layer-level checks
// ---------------------------------------------------------------------------
static smg_status layer_shape_ok(int c_in, int c_out, int n, int h, int w) {
  if (c_in < 8 || c_in % 8 || c_in > 64) return nfail(SMG_EINVAL, "c_in must be a multiple of 8 in [8, 64]");
  if (c_out != 32) return nfail(SMG_EINVAL, "c_out must be 32");
  if (n < 1 || h < 1 || w < 1) return nfail(SMG_EINVAL, "image batch must be non-empty");
  return SMG_OK;
}

extern "C" smg_status smg_net_conv3(const unsigned short* x, int c_in, const unsigned short* W, const float* b,
                                    unsigned short* y, int c_out, int relu, int n, int h, int w, void* stream) {
  NST(layer_shape_ok(c_in, c_out, n, h, w));
  if (!x || !W || !y) return nfail(SMG_EINVAL, "x, W and y must not be NULL");
  NCHK(smgn::conv3(x, c_in, c_in, W, b, y, c_out, c_out, nullptr, 0, relu != 0, n, h, w,
                   static_cast<hipStream_t>(stream)));
  return SMG_OK;
}

extern "C" size_t smg_net_conv3_wgrad_work_bytes(int c_in, int c_out, int n, int h, int w) {
  if (layer_shape_ok(c_in, c_out, n, h, w) != SMG_OK) return 0;
  return sizeof(float) * smgn::wgrad_partials(n * h * w, c_out, c_in);
}

extern "C" smg_status smg_net_conv3_wgrad(const unsigned short* g, int c_out, const unsigned short* x, int c_in, float* dW,
                                          float* db, int n, int h, int w, void* work, size_t work_bytes, void* stream) {
  NST(layer_shape_ok(c_in, c_out, n, h, w));
  if (!g || !x || !dW || !db) return nfail(SMG_EINVAL, "g, x, dW and db must not be NULL");
  const size_t need = smg_net_conv3_wgrad_work_bytes(c_in, c_out, n, h, w);
  if (!work || work_bytes < need) return nfail(SMG_EWORKSPACE, strprintf("wgrad work buffer of %zu bytes needed", need));
  hipStream_t st = static_cast<hipStream_t>(stream);
  NCHK(smgn::fill_f32(db, c_out, 0.f, st));
  NCHK(smgn::wgrad(g, c_out, c_out, x, c_in, c_in, static_cast<float*>(work), work_bytes / sizeof(float), dW, db, n, h, w,
                   st));
  return SMG_OK;
}

// ---------------------------------------------------------------------------
// weight gradient without allocation: the partial sums live in a static
// device array (one per GPU, held until the process ends)
// ---------------------------------------------------------------------------
namespace {

static __device__ __align__(256) float scratch[smgn::kWgradMaxPartials];

constexpr int kMaxDevices = 64;
// most pixels a call accepts: keeps every pixel index of the kernels in int range
constexpr long long kNoAllocMaxPixels = 1LL << 28;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's scratch array (looked up once per device,
// with that device current).
smg_status scratch_of_current_device(float** out) {
  int dev = 0;
  NCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return nfail(SMG_EINVAL, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return nfail(SMG_EHIP, strprintf("hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e)));
    g_scratch_ptr[dev] = static_cast<float*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return SMG_OK;
}

}  // namespace

extern "C" smg_status smg_net_conv3_wgrad_noalloc(const unsigned short* g, int c_out, const unsigned short* x, int c_in,
                                                  float* dW, float* db, int n, int h, int w, void* stream) {
  NST(layer_shape_ok(c_in, c_out, n, h, w));
  if (!g || !x || !dW || !db) return nfail(SMG_EINVAL, "g, x, dW and db must not be NULL");
  if ((long long)n * h * w > kNoAllocMaxPixels)
    return nfail(SMG_EINVAL, strprintf("n*h*w = %lld pixels exceeds the no-allocation limit of %lld",
                                       (long long)n * h * w, kNoAllocMaxPixels));
  const size_t need = smgn::wgrad_partials(n * h * w, c_out, c_in);
  if (need > smgn::kWgradMaxPartials)
    return nfail(SMG_EINVAL, strprintf("partial sums of %zu floats exceed the %zu-float scratch", need,
                                       smgn::kWgradMaxPartials));
  float* part = nullptr;
  NST(scratch_of_current_device(&part));
  hipStream_t st = static_cast<hipStream_t>(stream);
  NCHK(smgn::fill_f32(db, c_out, 0.f, st));
  NCHK(smgn::wgrad(g, c_out, c_out, x, c_in, c_in, part, smgn::kWgradMaxPartials, dW, db, n, h, w, st));
  return SMG_OK;
}
