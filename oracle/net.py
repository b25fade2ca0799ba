"""The learned initial guess -- oracle side (test infrastructure only).

A small per-mode 2D convolutional network predicts how a low-m mode plane
of the potential changes from one time step to the next.  The input is one
real plane (the real or imaginary part of a mode) with eight channels,
  0: f_t / s_f              (this step's right-hand side)
  1: (f_t - f_{t-1}) / s_d  (its change since the previous step)
  2: u_{t-1} / s_u          (the previous step's solution)
  3: m / 4                  (the azimuthal index),
  4, 5: (i + 1/2) / n_a - 1/2, (j + 1/2) / n_b - 1/2  (the position on the grid),
  6: (u_{t-1} - u_{t-2}) / s_o  (this part of the previous step's change,
     of unit RMS since s_o is then its RMS),
  7: the same part of -i (u_{t-1} - u_{t-2}) / s_o  (the other part, with
     the sign a rotation of the mode gives: a rotation by a small angle a
     changes the mode by a times -i m u; zero for m = 0),
  channels 6 and 7 are zero when there is no solution two steps back or the
  plane is static,
and the output is (u_t - u_{t-1}) / s_o, so that the guess is
u_{t-1} + s_o * net(x).  s_f, s_d and s_u are the per-plane RMS values of
f_t, f_t - f_{t-1} and u_{t-1}; s_o is the RMS of u_{t-1} - u_{t-2} when
that exists, else s_u s_d / s_f.  The output
layer starts at zero: the untrained network reproduces the previous-step
warm start exactly.

Architecture (a U-Net with 4 levels and 32 channels): at each encoder level
two 3x3 convolutions with ReLU (zero padding), 2x2 average pooling between
levels; in the decoder nearest-neighbour upsampling by 2, concatenation
[upsampled, encoder output] (64 channels), two 3x3 convolutions with ReLU;
a final 1x1 convolution to one channel without activation.

Arithmetic convention (shared with the HIP kernels): weights and every
stored activation and activation gradient are BF16 (round to nearest even,
from the FP32 value the accumulator holds); sums accumulate in FP32 on the
GPU and in FP64 here; weight gradients, biases, the output and the loss are
FP32/FP64.  Rounding points (``rounding=True``):
  conv output (after bias and ReLU) -> BF16; pooling output -> BF16;
  upsampling copies BF16; the network output stays unrounded;
  backward: the gradient entering a layer's input -> BF16 (after the ReLU
  mask of that input, and after summing the skip and pooling paths).
With ``rounding=False`` everything is FP64 (used by the finite-difference
pins of the backward pass).

Layout: activations are NHWC arrays (N, H, W, C); a 3x3 weight tensor is
(C_out, 9, C_in) with tap t = 3 (dy + 1) + (dx + 1) reading input pixel
(y + dy, x + dx); the parameter vector concatenates, layer by layer, the
weights then the biases.
"""
import numpy as np

LEVELS = 4
CH = 32
IN_CH = 8
# a plane whose last change is below this fraction of its RMS is static (the
# previous solution is already a better start than a guess needs to be): no
# extrapolation, correction or target
STATIC = 1e-4


def layer_shapes(levels=LEVELS, ch=CH, in_ch=IN_CH):
    """(kind, c_in, c_out) of every layer in parameter order."""
    shapes = []
    cin = in_ch
    for _ in range(levels):            # encoder (the last level is the bottom)
        shapes += [("conv3", cin, ch), ("conv3", ch, ch)]
        cin = ch
    for _ in range(levels - 1):        # decoder
        shapes += [("conv3", 2 * ch, ch), ("conv3", ch, ch)]
    shapes.append(("conv1", ch, 1))
    return shapes


def n_params(levels=LEVELS, ch=CH, in_ch=IN_CH):
    n = 0
    for kind, ci, co in layer_shapes(levels, ch, in_ch):
        n += co * ci * (9 if kind == "conv3" else 1) + co
    return n


def unpack(params, levels=LEVELS, ch=CH, in_ch=IN_CH):
    """List of (W, b) per layer; W is (c_out, 9, c_in) or (c_out, c_in)."""
    out, k = [], 0
    for kind, ci, co in layer_shapes(levels, ch, in_ch):
        nw = co * ci * (9 if kind == "conv3" else 1)
        W = params[k:k + nw].reshape((co, 9, ci) if kind == "conv3" else (co, ci))
        k += nw
        b = params[k:k + co]
        k += co
        out.append((W, b))
    return out


def pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


# -- BF16 ---------------------------------------------------------------------
def bf16(x):
    """Round to the nearest BF16 value (ties to even) via the FP32 value."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(f)
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def _q(x, rounding):
    return bf16(x) if rounding else x


# -- layers --------------------------------------------------------------------
def _shift(x, dy, dx):
    """y[n, i, j] = x[n, i + dy, j + dx] with zeros outside."""
    N, H, W, C = x.shape
    y = np.zeros_like(x)
    i0, i1 = max(0, -dy), min(H, H - dy)
    j0, j1 = max(0, -dx), min(W, W - dx)
    y[:, i0:i1, j0:j1] = x[:, i0 + dy:i1 + dy, j0 + dx:j1 + dx]
    return y


TAPS = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def conv3(x, W, b):
    """3x3 'same' correlation: out[.., o] = b[o] + sum_{t, c} W[o, t, c] x[.. + tap t, c]."""
    out = np.zeros(x.shape[:3] + (W.shape[0],))
    for t, (dy, dx) in enumerate(TAPS):
        out += np.tensordot(_shift(x, dy, dx), W[:, t, :], axes=([3], [1]))
    return out + b


def conv3_backward(x, W, g):
    """Gradients of sum(g * conv3(x, W, b)) w.r.t. x, W, b."""
    gx = np.zeros_like(x)
    gW = np.zeros_like(W)
    for t, (dy, dx) in enumerate(TAPS):
        xs = _shift(x, dy, dx)
        gW[:, t, :] = np.tensordot(g, xs, axes=([0, 1, 2], [0, 1, 2]))
        gx += _shift(np.tensordot(g, W[:, t, :], axes=([3], [0])), -dy, -dx)
    gb = g.sum(axis=(0, 1, 2))
    return gx, gW, gb


def pool2(x):
    N, H, W, C = x.shape
    return x.reshape(N, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def pool2_backward(g):
    return np.repeat(np.repeat(g, 2, axis=1), 2, axis=2) / 4.0


def up2(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up2_backward(g):
    N, H, W, C = g.shape
    return g.reshape(N, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


# -- network -------------------------------------------------------------------
def forward(params, x, rounding=True, levels=LEVELS, ch=CH):
    """Network output (N, H, W) and the cache of the backward pass."""
    L = unpack(params, levels, ch, x.shape[3])
    q = lambda v: _q(v, rounding)
    Lq = [(q(W), b) for W, b in L] if rounding else L
    cache = {"x": x, "L": Lq, "enc": [], "dec": [], "rounding": rounding}
    h = q(x)
    k = 0
    enc_out = []
    for lev in range(levels):
        if lev > 0:
            h = q(pool2(enc_out[-1]))
        a = q(np.maximum(conv3(h, *Lq[k]), 0.0))
        e = q(np.maximum(conv3(a, *Lq[k + 1]), 0.0))
        cache["enc"].append((h, a, e))
        enc_out.append(e)
        k += 2
    d = enc_out[-1]
    for lev in range(levels - 2, -1, -1):
        cat = np.concatenate([up2(d), enc_out[lev]], axis=3)
        a = q(np.maximum(conv3(cat, *Lq[k]), 0.0))
        d = q(np.maximum(conv3(a, *Lq[k + 1]), 0.0))
        cache["dec"].append((cat, a, d))
        k += 2
    W1, b1 = Lq[k]
    out = np.tensordot(d, W1, axes=([3], [1]))[..., 0] + b1[0]
    cache["d0"] = d
    return out, cache


def backward(params, cache, g_out, levels=LEVELS, ch=CH):
    """Gradient of sum(g_out * out) w.r.t. the parameters (packed vector)."""
    rounding = cache["rounding"]
    q = lambda v: _q(v, rounding)
    Lq = cache["L"]
    grads = [None] * len(Lq)
    k = len(Lq) - 1
    W1, _ = Lq[k]
    d = cache["d0"]
    g = g_out[..., None]
    grads[k] = (np.tensordot(g, d, axes=([0, 1, 2], [0, 1, 2])), g.sum(axis=(0, 1, 2)))
    gd = q(np.tensordot(g, W1, axes=([3], [0])) * (d > 0))
    k -= 1
    skip_g = [None] * levels
    for idx in range(len(cache["dec"]) - 1, -1, -1):   # from the output back
        lev = levels - 2 - idx                          # encoder level of the skip input
        cat, a, dd = cache["dec"][idx]
        gx, gW, gb = conv3_backward(a, Lq[k][0], gd)
        grads[k] = (gW, gb)
        ga = q(gx * (a > 0))
        gx, gW, gb = conv3_backward(cat, Lq[k - 1][0], ga)
        grads[k - 1] = (gW, gb)
        k -= 2
        gcat = q(gx)
        skip_g[lev] = gcat[..., ch:]
        gup = gcat[..., :ch]
        below = cache["dec"][idx - 1][2] if idx > 0 else cache["enc"][levels - 1][2]
        gd = q(up2_backward(gup) * (below > 0))
    # encoder, bottom up: gd is the gradient at the bottom encoder output
    ge = gd
    for lev in range(levels - 1, -1, -1):
        h, a, e = cache["enc"][lev]
        gx, gW, gb = conv3_backward(a, Lq[k][0], ge)
        grads[k] = (gW, gb)
        ga = q(gx * (a > 0))
        gx, gW, gb = conv3_backward(h, Lq[k - 1][0], ga)
        grads[k - 1] = (gW, gb)
        k -= 2
        if lev > 0:
            eprev = cache["enc"][lev - 1][2]
            ge = q((q(pool2_backward(q(gx))) + skip_g[lev - 1]) * (eprev > 0))
    return pack(grads)


def loss(out, target):
    """Mean squared error and its gradient w.r.t. the output."""
    diff = out - target
    n = diff.size
    return float(np.sum(diff * diff) / n), 2.0 * diff / n


# -- the learned guess inside a solve -------------------------------------------
# The network is this build's addition to the paper's warm start (Sec. 5.1:
# each multigrid solve starts from the previous time step's solution).  For
# the low modes 0..m_max the solve may instead start from
#   cand = u_{t-1} + (u_{t-1} - u_{t-2}) + s_o * net(x)
# (the linear extrapolation of the last two solutions plus the network's
# correction; without u_{t-2}, u_{t-1} + s_o * net(x)), whichever of cand
# and u_{t-1} has the smaller volume-weighted defect norm after one
# smoothing step of each (the multigrid removes the rough part of any error
# in its first sweep; what is left decides the cycle count).  The network
# is trained on the correction the candidate needs,
# (u_t - u_{t-1} - (u_{t-1} - u_{t-2})) / s_o.
def image_mode(k):
    """Real image k -> (mode m, part): 0 -> (0, real); 2m - 1 -> (m, real);
    2m -> (m, imaginary)."""
    m = (k + 1) // 2
    return m, (1 if (k > 0 and k % 2 == 0) else 0)


def _part(z, im):
    return z.imag if im else z.real


def guess_images(f, fprev, uprev, m_max, uprev2=None):
    """Network inputs and scales of modes 0..m_max.

    f, fprev, uprev: complex (>= m_max + 1, n_a, n_b) planes of this step's
    right-hand side, the previous step's and the previous solution; uprev2
    (optional) the solution of the step before that.  Returns
    x (2 m_max + 1, n_a, n_b, 8) and sc (2 m_max + 1, 4) = (s_f, s_d, s_u,
    s_o) per image, the RMS values of f, f - fprev and uprev over the plane
    (1 where zero) and the output scale s_o: the RMS of uprev - uprev2 when
    uprev2 is given (the size of the last change; 0 marks a static plane,
    one whose change is below STATIC of its RMS), else s_u s_d / s_f."""
    n_img = 2 * m_max + 1
    na, nb = f.shape[1], f.shape[2]
    x = np.zeros((n_img, na, nb, 8))
    sc = np.zeros((n_img, 4))
    ci = (np.arange(na) + 0.5) / na - 0.5
    cj = (np.arange(nb) + 0.5) / nb - 0.5
    for k in range(n_img):
        m, im = image_mode(k)
        fv, fp, uv = _part(f[m], im), _part(fprev[m], im), _part(uprev[m], im)
        s = [float(np.sqrt(np.mean(v * v))) for v in (fv, fv - fp, uv)]
        s = [v if v > 0.0 else 1.0 for v in s]
        so = s[2] * s[1] / s[0]
        if uprev2 is not None:
            e = uv - _part(uprev2[m], im)
            so = float(np.sqrt(np.mean(e * e)))
            so = so if so > STATIC * s[2] else 0.0      # static plane: marked by s_o = 0
        sc[k] = (s[0], s[1], s[2], so)
        x[k, :, :, 0] = fv / s[0]
        x[k, :, :, 1] = (fv - fp) / s[1]
        x[k, :, :, 2] = uv / s[2]
        x[k, :, :, 3] = m / 4.0
        x[k, :, :, 4] = ci[:, None]
        x[k, :, :, 5] = cj[None, :]
        if uprev2 is not None and sc[k, 3] > 0.0:
            d = (uprev[m] - uprev2[m]) / sc[k, 3]
            x[k, :, :, 6] = _part(d, im)
            if m > 0:
                x[k, :, :, 7] = _part(-1j * d, im)
    return x, sc


def guess_candidate(uprev, y, sc, m_max, uprev2=None):
    """cand = u_{t-1} + (u_{t-1} - u_{t-2}) + s_o y per real image (no
    extrapolation without uprev2; the imaginary part of m = 0 is only
    extrapolated)."""
    cand = np.array(uprev[:m_max + 1], dtype=np.complex128)
    if uprev2 is not None:
        for m in range(m_max + 1):
            kr = 0 if m == 0 else 2 * m - 1
            ki = kr if m == 0 else 2 * m            # m = 0: the imaginary part follows the real image
            d = cand[m] - np.asarray(uprev2[m], dtype=np.complex128)
            cand[m] = cand[m] + (d.real if sc[kr, 3] > 0.0 else 0.0) + 1j * (d.imag if sc[ki, 3] > 0.0 else 0.0)
    for k in range(2 * m_max + 1):
        m, im = image_mode(k)
        if im:
            cand[m] = cand[m] + 1j * sc[k, 3] * y[k]
        else:
            cand[m] = cand[m] + sc[k, 3] * y[k]
    return cand


def guess_base(uprev, sc, m_max, uprev2=None):
    """The start the judge weighs the candidate against: the candidate
    without the network's correction, u_{t-1} + (u_{t-1} - u_{t-2}) on the
    parts that change (u_{t-1} without uprev2 or on static parts)."""
    return guess_candidate(uprev, np.zeros((2 * m_max + 1,) + np.shape(uprev)[1:]), sc, m_max, uprev2=uprev2)


def guess_target(u, uprev, sc, m_max, uprev2=None):
    """The training target of each real image: the correction the candidate
    needs to become u_t, (u_t - u_{t-1} - (u_{t-1} - u_{t-2})) / s_o."""
    out = np.zeros((2 * m_max + 1,) + u.shape[1:])
    for k in range(2 * m_max + 1):
        m, im = image_mode(k)
        d = _part(u[m], im) - _part(uprev[m], im)
        if uprev2 is not None:
            d = d - (_part(uprev[m], im) - _part(uprev2[m], im))
        out[k] = d / sc[k, 3] if sc[k, 3] > 0.0 else 0.0
    return out


def guess_judge(level, f, cand, uprev, m_max, n_sor=2, line_solver="sor"):
    """Per mode m <= m_max: 1 where the candidate's defect norm after one
    smoothing step (``level``: an oracle.multigrid.MGLevel of the finest
    grid) is below that of the other start ``uprev`` (in a solve: the
    baseline of guess_base).  Returns (used, norm of the candidate, norm of
    the other start)."""
    used = np.zeros(m_max + 1, dtype=int)
    nc = np.zeros(m_max + 1)
    nu = np.zeros(m_max + 1)
    for m in range(m_max + 1):
        norms = []
        for u0 in (cand[m], uprev[m]):
            u = np.array(u0, dtype=np.complex128)
            if line_solver == "exact":
                level.smooth_exact(u, f[m], m)
            else:
                level.smooth(u, f[m], m, n_sor)
            norms.append(float(level.op.norm_v(f[m] - level.apply(u, m))))
        nc[m], nu[m] = norms
        used[m] = 1 if norms[0] < norms[1] else 0
    return used, nc, nu
