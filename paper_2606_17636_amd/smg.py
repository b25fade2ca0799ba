"""ctypes binding of libsmg.so (include/smg.h): argument marshalling only.

Every step of the solve runs in the HIP library; torch is used for device
memory (the workspace and the caller's arrays) and for the current stream.
Loading fails loudly if the library has not been built -- there is no
fallback path.
"""
import ctypes
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsmg.so")

SPHERICAL, CYLINDRICAL = 0, 1
UNIFORM, LOG = 0, 1
FP64, MIXED = 0, 1
DGF_AUTO, DGF_AUX, DGF_EXTENDED = 0, 1, 2
LINE_SOR, LINE_EXACT = 0, 1
NU_AUTO = -1  # nu_pre = nu_post = NU_AUTO: smoothing steps chosen at setup
LAUNCH_GRAPH, LAUNCH_DYNAMIC = 0, 1
COARSE_EXACT, COARSE_SOR = 0, 1
WARM_PREV = 1
TIMINGS = 2
NET_GUESS = 4
WARM_EXTRAP = 8

STATUS = {0: "SMG_OK", -1: "SMG_EINVAL", -2: "SMG_ENOCONV", -3: "SMG_EHIP", -4: "SMG_EWORKSPACE", -5: "SMG_ESTATE"}


class SmgError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class Grid(ctypes.Structure):
    _fields_ = [("geometry", ctypes.c_int), ("radial", ctypes.c_int), ("n_a", ctypes.c_int), ("n_b", ctypes.c_int),
                ("n_phi", ctypes.c_int), ("a_min", ctypes.c_double), ("a_max", ctypes.c_double),
                ("b_min", ctypes.c_double), ("b_max", ctypes.c_double), ("G", ctypes.c_double)]


class Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("nu_pre", ctypes.c_int), ("nu_post", ctypes.c_int),
                ("n_sor", ctypes.c_int), ("max_cycles", ctypes.c_int), ("dgf_method", ctypes.c_int),
                ("n_pad", ctypes.c_int), ("dgf_tol", ctypes.c_double), ("line_solver", ctypes.c_int),
                ("launch", ctypes.c_int), ("autotune", ctypes.c_int), ("coarse_cells", ctypes.c_int),
                ("coarse_solver", ctypes.c_int), ("warm_extrapolate", ctypes.c_int)]


_PI = ctypes.POINTER(ctypes.c_int)
_PD = ctypes.POINTER(ctypes.c_double)


class Info(ctypes.Structure):
    _fields_ = [("n_modes", ctypes.c_int), ("cycles1", _PI), ("cycles2", _PI), ("resid1", _PD), ("resid2", _PD),
                ("total_cycles", ctypes.c_int), ("converged", ctypes.c_int), ("ms_fft", ctypes.c_double),
                ("ms_mg1", ctypes.c_double), ("ms_james", ctypes.c_double), ("ms_mg2", ctypes.c_double),
                ("ms_ifft", ctypes.c_double)]


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char_p), ("launches", ctypes.c_int), ("total_ms", ctypes.c_double),
                ("bytes", ctypes.c_double)]


_lib = None
_VP = ctypes.c_void_p


def load():
    """Load libsmg.so (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} not built: run `python -m paper_2606_17636_amd.build`")
    # torch brings its own HIP runtime (soname libamdhip64.so.7); importing it
    # first makes libsmg.so bind to that same runtime instead of loading a
    # second copy from /opt/rocm, which could not share the device with it.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P = _VP
    sig = {
        "smg_plan_create": ([ctypes.POINTER(Grid), ctypes.POINTER(Opts), ctypes.POINTER(P)], ctypes.c_int),
        "smg_workspace_bytes": ([P], ctypes.c_size_t),
        "smg_plan_setup": ([P, P, ctypes.c_size_t, P], ctypes.c_int),
        "smg_solve": ([P, P, P, ctypes.c_double, ctypes.c_uint, P, ctypes.POINTER(Info)], ctypes.c_int),
        "smg_plan_destroy": ([P], ctypes.c_int),
        "smg_last_error": ([], ctypes.c_char_p),
        "smg_plan_geometry": ([P, _PD, _PD, _PD, _PD], ctypes.c_int),
        "smg_plan_shape": ([P, _PI, _PI, _PI, _PI], ctypes.c_int),
        "smg_fft_forward": ([P, P, P, P], ctypes.c_int),
        "smg_fft_inverse": ([P, P, P, P], ctypes.c_int),
        "smg_mg_solve": ([P, P, P, ctypes.c_double, P, _PI, _PD], ctypes.c_int),
        "smg_mg_vcycle": ([P, P, P, P], ctypes.c_int),
        "smg_mg_smooth": ([P, P, P, P], ctypes.c_int),
        "smg_mg_residual": ([P, P, P, P, P], ctypes.c_int),
        "smg_james": ([P, P, P, P, P, P, P], ctypes.c_int),
        "smg_acceleration": ([P, P, P, P, P, P, P], ctypes.c_int),
        "smg_dgf_table": ([P, ctypes.c_int, _PD, P], ctypes.c_int),
        "smg_profile_begin": ([P], ctypes.c_int),
        "smg_profile_end": ([P, ctypes.POINTER(KernelStat), ctypes.c_int, _PI], ctypes.c_int),
        "smg_tune_report": ([P], ctypes.c_char_p),
        "smg_batch_create": ([ctypes.POINTER(P), ctypes.c_int, ctypes.POINTER(P)], ctypes.c_int),
        "smg_batch_workspace_bytes": ([P], ctypes.c_size_t),
        "smg_batch_setup": ([P, P, ctypes.c_size_t, P], ctypes.c_int),
        "smg_batch_solve": ([P, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.c_double, ctypes.c_uint, P,
                             ctypes.POINTER(Info)], ctypes.c_int),
        "smg_batch_tune_report": ([P], ctypes.c_char_p),
        "smg_batch_destroy": ([P], ctypes.c_int),
        "smg_plan_net_work_bytes": ([P, P, ctypes.c_int], ctypes.c_size_t),
        "smg_plan_attach_net": ([P, P, ctypes.c_int, P, ctypes.c_size_t, P], ctypes.c_int),
        "smg_plan_record": ([P, P, ctypes.c_int, P], ctypes.c_int),
        "smg_plan_recorded": ([P, P], ctypes.c_int),
        "smg_plan_net_used": ([P, _PI, P], ctypes.c_int),
        "smg_net_guess_step": ([P, ctypes.c_int, P, P, P, P, P, P, P, _PI, P], ctypes.c_int),
        "smg_net_conv3": ([P, ctypes.c_int, P, P, P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                           ctypes.c_int, P], ctypes.c_int),
        "smg_net_conv3_wgrad_work_bytes": ([ctypes.c_int] * 5, ctypes.c_size_t),
        "smg_net_conv3_wgrad": ([P, ctypes.c_int, P, ctypes.c_int, P, P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P,
                                 ctypes.c_size_t, P], ctypes.c_int),
        "smg_net_conv3_wgrad_noalloc": ([P, ctypes.c_int, P, ctypes.c_int, P, P, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int, P], ctypes.c_int),
        "smg_net_create": ([ctypes.c_int, ctypes.c_int, ctypes.POINTER(P)], ctypes.c_int),
        "smg_net_destroy": ([P], ctypes.c_int),
        "smg_net_param_count": ([P], ctypes.c_longlong),
        "smg_net_state_bytes": ([P], ctypes.c_size_t),
        "smg_net_bind": ([P, P, ctypes.c_size_t, P], ctypes.c_int),
        "smg_net_set_params": ([P, P, P], ctypes.c_int),
        "smg_net_get_params": ([P, P, P], ctypes.c_int),
        "smg_net_get_grads": ([P, P, P], ctypes.c_int),
        "smg_net_work_bytes": ([P, ctypes.c_int, ctypes.c_int, ctypes.c_int], ctypes.c_size_t),
        "smg_net_forward": ([P, P, P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, ctypes.c_size_t, P], ctypes.c_int),
        "smg_net_backward": ([P, P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, ctypes.c_size_t, P], ctypes.c_int),
        "smg_net_train_step": ([P, P, ctypes.c_int, _PI, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_float, P,
                                ctypes.c_size_t, P, ctypes.POINTER(ctypes.c_float)], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(status, ok=(0,)):
    if status not in ok:
        raise SmgError(status, load().smg_last_error().decode())
    return status


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(a):
    return a.ctypes.data_as(_PD)


def _iptr(a):
    return a.ctypes.data_as(_PI)


class Plan:
    """One grid + options.  Host tables are built at construction; call
    ``setup()`` to bind a device workspace and build the DGF tables."""

    def __init__(self, geometry, radial, n_a, n_b, n_phi, a_min, a_max, b_min, b_max, G=1.0, precision=FP64,
                 nu_pre=2, nu_post=2, n_sor=2, max_cycles=60, dgf_method=DGF_AUTO, n_pad=16, dgf_tol=1e-13,
                 line_solver=LINE_SOR, launch=LAUNCH_GRAPH, autotune=False, coarse_cells=0, coarse_solver=COARSE_EXACT,
                 warm_extrapolate=False):
        lib = load()
        geo = {"spherical": SPHERICAL, "cylindrical": CYLINDRICAL}.get(geometry, geometry)
        rad = {"uniform": UNIFORM, "log": LOG}.get(radial, radial)
        prec = {"fp64": FP64, "mixed": MIXED}.get(precision, precision)
        self.grid = Grid(geo, rad, n_a, n_b, n_phi, a_min, a_max, b_min, b_max, G)
        ls = {"sor": LINE_SOR, "exact": LINE_EXACT}.get(line_solver, line_solver)
        lc = {"graph": LAUNCH_GRAPH, "dynamic": LAUNCH_DYNAMIC}.get(launch, launch)
        cs = {"exact": COARSE_EXACT, "sor": COARSE_SOR}.get(coarse_solver, coarse_solver)
        self.opts = Opts(prec, nu_pre, nu_post, n_sor, max_cycles, dgf_method, n_pad, dgf_tol, ls, lc,
                         1 if autotune else 0, coarse_cells, cs, int(warm_extrapolate))
        self.line_solver = ls
        self._h = ctypes.c_void_p()
        _check(lib.smg_plan_create(ctypes.byref(self.grid), ctypes.byref(self.opts), ctypes.byref(self._h)))
        self.n_a, self.n_b, self.n_phi = n_a, n_b, n_phi
        self.n_modes = n_phi // 2 + 1
        self.workspace_bytes = int(lib.smg_workspace_bytes(self._h))
        nl, ng = ctypes.c_int(), ctypes.c_int()
        la = (ctypes.c_int * 16)()
        lb = (ctypes.c_int * 16)()
        _check(lib.smg_plan_shape(self._h, ctypes.byref(nl), ctypes.byref(ng), la, lb))
        self.n_levels, self.n_ghost = nl.value, ng.value
        self.level_shapes = [(la[i], lb[i]) for i in range(nl.value)]
        self._ws = None

    def __del__(self):
        if getattr(self, "_h", None) and self._h.value and _lib is not None:
            _lib.smg_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    @property
    def handle(self):
        return self._h

    # -- host queries -------------------------------------------------------
    def geometry(self):
        """Cell centres (a, b, phi) and volumes dv[n_a, n_b] as numpy arrays."""
        a = np.zeros(self.n_a)
        b = np.zeros(self.n_b)
        p = np.zeros(self.n_phi)
        dv = np.zeros((self.n_a, self.n_b))
        _check(load().smg_plan_geometry(self._h, _dptr(a), _dptr(b), _dptr(p), _dptr(dv)))
        return a, b, p, dv

    # -- device -------------------------------------------------------------
    def setup(self, device="cuda"):
        import torch
        self._ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=device)
        base = self._ws.data_ptr()
        off = (-base) % 256
        _check(load().smg_plan_setup(self._h, ctypes.c_void_p(base + off), ctypes.c_size_t(self.workspace_bytes),
                                     _stream()))
        return self

    def _f64(self, t, shape):
        import torch
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and tuple(t.shape) == tuple(shape)):
            raise ValueError(f"expected a contiguous cuda float64 tensor of shape {shape}, got "
                             f"{tuple(t.shape)} {t.dtype} {t.device}")
        return t

    def _c128(self, t, shape):
        import torch
        if not (t.is_cuda and t.dtype == torch.complex128 and t.is_contiguous() and tuple(t.shape) == tuple(shape)):
            raise ValueError(f"expected a contiguous cuda complex128 tensor of shape {shape}")
        return t

    # -- learned guess ---------------------------------------------------------
    def attach_net(self, net, m_max=4):
        """Use `net` (an smg.Net) for the guess of modes 0..m_max (None detaches)."""
        lib = load()
        if net is None:
            _check(lib.smg_plan_attach_net(self._h, None, 0, None, ctypes.c_size_t(0), _stream()))
            self._net = None
            return self
        nb = int(lib.smg_plan_net_work_bytes(self._h, net.handle, m_max))
        if nb == 0:
            raise SmgError(-1, "network does not fit this grid")
        self._net_work, ptr = _aligned(nb, net.device)
        _check(lib.smg_plan_attach_net(self._h, net.handle, m_max, ctypes.c_void_p(ptr), ctypes.c_size_t(nb), _stream()))
        self._net = net
        self.m_max = m_max
        return self

    def record(self, samples, capacity):
        """Append training samples of later warm solves to `samples` (float32 cuda)."""
        _check(load().smg_plan_record(self._h, _ptr(samples) if samples is not None else None, int(capacity), _stream()))

    def recorded(self):
        return int(load().smg_plan_recorded(self._h, _stream()))

    def net_used(self):
        used = np.zeros(2 * (self.m_max + 1), dtype=np.int32)
        _check(load().smg_plan_net_used(self._h, _iptr(used), _stream()))
        return used.reshape(2, self.m_max + 1)

    def net_guess_step(self, t, f, fprev, uprev, uprev2=None):
        """The learned-guess step of solve t on caller planes (complex128
        cuda, shape (m_max+1, n_a, n_b)): returns (guess, x, y, used)."""
        import torch
        shape = (self.m_max + 1, self.n_a, self.n_b)
        for a in (f, fprev, uprev) + ((uprev2,) if uprev2 is not None else ()):
            self._c128(a, shape)
        n_img = 2 * self.m_max + 1
        guess = torch.empty(shape, dtype=torch.complex128, device=f.device)
        x = torch.empty((n_img, self.n_a, self.n_b, 8), dtype=torch.float32, device=f.device)
        y = torch.empty((n_img, self.n_a, self.n_b), dtype=torch.float32, device=f.device)
        used = np.zeros(self.m_max + 1, dtype=np.int32)
        _check(load().smg_net_guess_step(self._h, int(t), _ptr(f), _ptr(fprev), _ptr(uprev), _ptr(uprev2), _ptr(guess),
                                         _ptr(x), _ptr(y), _iptr(used), _stream()))
        return guess, x, y, used

    def solve(self, rho, tol=1e-8, warm=False, out=None, timings=False, allow_noconv=False, net=False,
              extrapolate=False):
        """Phi for the density rho (cuda float64 [n_a, n_b, n_phi]); returns
        (phi, info dict).  extrapolate: warm start from the linear
        extrapolation of the last two solutions (plan made with
        warm_extrapolate=True)."""
        import torch
        shape = (self.n_a, self.n_b, self.n_phi)
        self._f64(rho, shape)
        phi = out if out is not None else torch.empty(shape, dtype=torch.float64, device=rho.device)
        self._f64(phi, shape)
        M = self.n_modes
        c1 = np.zeros(M, dtype=np.int32)
        c2 = np.zeros(M, dtype=np.int32)
        r1 = np.zeros(M)
        r2 = np.zeros(M)
        info = Info(M, _iptr(c1), _iptr(c2), _dptr(r1), _dptr(r2), 0, 0, 0, 0, 0, 0, 0)
        flags = ((WARM_PREV if warm else 0) | (TIMINGS if timings else 0) | (NET_GUESS if net else 0) |
                 (WARM_EXTRAP if extrapolate else 0))
        st = load().smg_solve(self._h, _ptr(rho), _ptr(phi), ctypes.c_double(tol), ctypes.c_uint(flags), _stream(),
                              ctypes.byref(info))
        _check(st, ok=(0, -2) if allow_noconv else (0,))
        d = dict(cycles1=c1, cycles2=c2, resid1=r1, resid2=r2, total_cycles=info.total_cycles,
                 converged=bool(info.converged), status=st)
        if timings:
            d.update(ms_fft=info.ms_fft, ms_mg1=info.ms_mg1, ms_james=info.ms_james, ms_mg2=info.ms_mg2,
                     ms_ifft=info.ms_ifft)
        return phi, d

    def solve_nosync(self, rho, phi, tol=1e-8, warm=False, net=False, extrapolate=False):
        """smg_solve without the info report (for timing loops)."""
        flags = (WARM_PREV if warm else 0) | (NET_GUESS if net else 0) | (WARM_EXTRAP if extrapolate else 0)
        _check(load().smg_solve(self._h, _ptr(rho), _ptr(phi), ctypes.c_double(tol), ctypes.c_uint(flags), _stream(),
                                None))

    # -- steps ----------------------------------------------------------------
    def mode_shape(self):
        return (self.n_modes, self.n_a, self.n_b)

    def fft_forward(self, rho, out=None):
        import torch
        self._f64(rho, (self.n_a, self.n_b, self.n_phi))
        out = out if out is not None else torch.empty(self.mode_shape(), dtype=torch.complex128, device=rho.device)
        _check(load().smg_fft_forward(self._h, _ptr(rho), _ptr(self._c128(out, self.mode_shape())), _stream()))
        return out

    def fft_inverse(self, modes, out=None):
        import torch
        self._c128(modes, self.mode_shape())
        out = out if out is not None else torch.empty((self.n_a, self.n_b, self.n_phi), dtype=torch.float64,
                                                      device=modes.device)
        _check(load().smg_fft_inverse(self._h, _ptr(modes), _ptr(out), _stream()))
        return out

    def mg_solve(self, f, u, tol):
        self._c128(f, self.mode_shape())
        self._c128(u, self.mode_shape())
        cyc = np.zeros(self.n_modes, dtype=np.int32)
        res = np.zeros(self.n_modes)
        _check(load().smg_mg_solve(self._h, _ptr(f), _ptr(u), ctypes.c_double(tol), _stream(), _iptr(cyc), _dptr(res)))
        return cyc, res

    def mg_vcycle(self, f, u):
        _check(load().smg_mg_vcycle(self._h, _ptr(self._c128(f, self.mode_shape())),
                                    _ptr(self._c128(u, self.mode_shape())), _stream()))

    def mg_smooth(self, f, u):
        _check(load().smg_mg_smooth(self._h, _ptr(self._c128(f, self.mode_shape())),
                                    _ptr(self._c128(u, self.mode_shape())), _stream()))

    def mg_residual(self, f, u, out=None):
        import torch
        out = out if out is not None else torch.empty(self.mode_shape(), dtype=torch.complex128, device=f.device)
        _check(load().smg_mg_residual(self._h, _ptr(self._c128(f, self.mode_shape())),
                                      _ptr(self._c128(u, self.mode_shape())), _ptr(out), _stream()))
        return out

    def james(self, psi, f):
        import torch
        M, ng = self.n_modes, self.n_ghost
        sigma = torch.empty((M, ng), dtype=torch.complex128, device=psi.device)
        theta = torch.empty((M, ng), dtype=torch.complex128, device=psi.device)
        f2 = torch.empty(self.mode_shape(), dtype=torch.complex128, device=psi.device)
        _check(load().smg_james(self._h, _ptr(self._c128(psi, self.mode_shape())),
                                _ptr(self._c128(f, self.mode_shape())), _ptr(sigma), _ptr(theta), _ptr(f2), _stream()))
        return sigma, theta, f2

    def acceleration(self, phi, theta=None, out=None):
        """g = -grad Phi on the faces: (g_a, g_b, g_phi) of shapes
        (n_a+1, n_b, n_phi), (n_a, n_b+1, n_phi), (n_a, n_b, n_phi).  theta:
        complex (n_modes, n_ghost) screening potential, or None for that of
        the last solve."""
        import torch
        na, nb, npf = self.grid.n_a, self.grid.n_b, self.grid.n_phi
        self._f64(phi, (na, nb, npf))
        if theta is not None:
            self._c128(theta, (self.n_modes, self.n_ghost))
        if out is None:
            kw = dict(dtype=torch.float64, device=phi.device)
            out = (torch.empty((na + 1, nb, npf), **kw), torch.empty((na, nb + 1, npf), **kw),
                   torch.empty((na, nb, npf), **kw))
        g_a, g_b, g_p = out
        self._f64(g_a, (na + 1, nb, npf))
        self._f64(g_b, (na, nb + 1, npf))
        self._f64(g_p, (na, nb, npf))
        _check(load().smg_acceleration(self._h, _ptr(phi), _ptr(theta), _ptr(g_a), _ptr(g_b), _ptr(g_p), _stream()))
        return g_a, g_b, g_p

    def profile_begin(self):
        _check(load().smg_profile_begin(self._h))

    def profile_end(self):
        """Per kernel class: launches, total ms, algorithmic bytes."""
        arr = (KernelStat * 32)()
        n = ctypes.c_int()
        _check(load().smg_profile_end(self._h, arr, 32, ctypes.byref(n)))
        return {arr[i].name.decode(): dict(launches=arr[i].launches, total_ms=arr[i].total_ms, bytes=arr[i].bytes)
                for i in range(min(n.value, 32))}

    def tune_report(self):
        return load().smg_tune_report(self._h).decode()

    def dgf_table(self, m):
        out = np.zeros((self.n_ghost, self.n_ghost))
        _check(load().smg_dgf_table(self._h, int(m), _dptr(out), _stream()))
        return out


class Batch:
    """Several set-up plans solved together (every multigrid launch covers
    the mode planes of all of them)."""

    def __init__(self, plans):
        lib = load()
        self.plans = list(plans)
        arr = (ctypes.c_void_p * len(self.plans))(*[p.handle.value for p in self.plans])
        self._h = ctypes.c_void_p()
        _check(lib.smg_batch_create(arr, len(self.plans), ctypes.byref(self._h)))
        self.workspace_bytes = int(lib.smg_batch_workspace_bytes(self._h))
        self._ws = None

    def __del__(self):
        if getattr(self, "_h", None) and self._h.value and _lib is not None:
            _lib.smg_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def setup(self, device="cuda"):
        import torch
        self._ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=device)
        base = self._ws.data_ptr()
        off = (-base) % 256
        _check(load().smg_batch_setup(self._h, ctypes.c_void_p(base + off), ctypes.c_size_t(self.workspace_bytes),
                                      _stream()))
        return self

    def tune_report(self):
        return load().smg_batch_tune_report(self._h).decode()

    def solve(self, rhos, tol=1e-8, warm=False, outs=None, timings=False, info=True, extrapolate=False):
        """phi for every plan's density; returns (phis, infos or None)."""
        import torch
        n = len(self.plans)
        outs = outs if outs is not None else [torch.empty_like(r) for r in rhos]
        for p, r, o in zip(self.plans, rhos, outs):
            shape = (p.n_a, p.n_b, p.n_phi)
            p._f64(r, shape)
            p._f64(o, shape)
        rp = (ctypes.c_void_p * n)(*[r.data_ptr() for r in rhos])
        op = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
        flags = (WARM_PREV if warm else 0) | (TIMINGS if timings else 0) | (WARM_EXTRAP if extrapolate else 0)
        infos = None
        keep = []
        if info:
            infos = (Info * n)()
            for q, p in enumerate(self.plans):
                M = p.n_modes
                arrs = [np.zeros(M, dtype=np.int32), np.zeros(M, dtype=np.int32), np.zeros(M), np.zeros(M)]
                keep.append(arrs)
                infos[q] = Info(M, _iptr(arrs[0]), _iptr(arrs[1]), _dptr(arrs[2]), _dptr(arrs[3]), 0, 0, 0, 0, 0, 0, 0)
        _check(load().smg_batch_solve(self._h, rp, op, ctypes.c_double(tol), ctypes.c_uint(flags), _stream(), infos))
        if not info:
            return outs, None
        res = []
        for q in range(n):
            c1, c2, r1, r2 = keep[q]
            res.append(dict(cycles1=c1, cycles2=c2, resid1=r1, resid2=r2, total_cycles=infos[q].total_cycles,
                            converged=bool(infos[q].converged)))
        return outs, res


def _aligned(nbytes, device):
    import torch
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf, buf.data_ptr() + off


class Net:
    """The learned-guess U-Net (state and work buffers are torch tensors)."""

    def __init__(self, levels=4, channels=32, device="cuda"):
        lib = load()
        self._h = ctypes.c_void_p()
        _check(lib.smg_net_create(levels, channels, ctypes.byref(self._h)))
        self.levels = levels
        self.device = device
        self.n_params = int(lib.smg_net_param_count(self._h))
        nb = int(lib.smg_net_state_bytes(self._h))
        self._state, ptr = _aligned(nb, device)
        _check(lib.smg_net_bind(self._h, ctypes.c_void_p(ptr), ctypes.c_size_t(nb), _stream()))
        self._work = {}

    def __del__(self):
        if getattr(self, "_h", None) and self._h.value and _lib is not None:
            _lib.smg_net_destroy(self._h)
            self._h = ctypes.c_void_p()

    @property
    def handle(self):
        return self._h

    def set_params(self, params):
        import torch
        t = torch.as_tensor(np.asarray(params, dtype=np.float32) if not hasattr(params, "data_ptr") else params,
                            dtype=torch.float32, device=self.device).contiguous()
        assert t.numel() == self.n_params
        _check(load().smg_net_set_params(self._h, _ptr(t), _stream()))

    def params(self):
        import torch
        t = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        _check(load().smg_net_get_params(self._h, _ptr(t), _stream()))
        return t

    def grads(self):
        import torch
        t = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        _check(load().smg_net_get_grads(self._h, _ptr(t), _stream()))
        return t

    def work(self, n, h, w):
        key = (n, h, w)
        if key not in self._work:
            nb = int(load().smg_net_work_bytes(self._h, n, h, w))
            if nb == 0:
                raise ValueError(f"invalid image batch shape {key}")
            self._work[key] = (nb,) + _aligned(nb, self.device)
        nb, _, ptr = self._work[key]
        return ctypes.c_void_p(ptr), ctypes.c_size_t(nb)

    def forward(self, x):
        import torch
        n, h, w, c = x.shape
        y = torch.empty((n, h, w), dtype=torch.float32, device=x.device)
        wp, wb = self.work(n, h, w)
        _check(load().smg_net_forward(self._h, _ptr(x.contiguous()), _ptr(y), n, h, w, wp, wb, _stream()))
        return y

    def backward(self, dy):
        n, h, w = dy.shape
        wp, wb = self.work(n, h, w)
        _check(load().smg_net_backward(self._h, _ptr(dy.contiguous()), n, h, w, wp, wb, _stream()))
        return self.grads()

    def train_step(self, samples, idx, h, w, lr):
        n = len(idx)
        ia = np.ascontiguousarray(np.asarray(idx, dtype=np.int32))
        wp, wb = self.work(n, h, w)
        loss = ctypes.c_float()
        n_samples = samples.numel() // (h * w * 9)
        _check(load().smg_net_train_step(self._h, _ptr(samples), n_samples, _iptr(ia), n, h, w, ctypes.c_float(lr), wp,
                                         wb, _stream(), ctypes.byref(loss)))
        return loss.value


def conv3_layer(x, w, b=None, relu=True):
    """One 3x3 convolution layer (smg_net_conv3).  x: int16 cuda tensor of
    BF16 bit patterns (n, h, w, c_in); w: int16 BF16 bits (32, 9, c_in); b:
    float32 (32,) or None.  Returns the BF16 bits (n, h, w, 32)."""
    import torch
    n, h, wd, cin = x.shape
    cout = w.shape[0]
    y = torch.empty((n, h, wd, cout), dtype=torch.int16, device=x.device)
    _check(load().smg_net_conv3(_ptr(x.contiguous()), cin, _ptr(w.contiguous()), _ptr(b), _ptr(y), cout,
                                1 if relu else 0, n, h, wd, _stream()))
    return y


def conv3_wgrad(g, x):
    """Parameter gradients of a 3x3 layer (smg_net_conv3_wgrad): g int16 BF16
    bits (n, h, w, 32), x int16 BF16 bits (n, h, w, c_in).  Returns (dW
    float32 (32, 9, c_in), db float32 (32,))."""
    import torch
    n, h, wd, cout = g.shape
    cin = x.shape[3]
    lib = load()
    nb = int(lib.smg_net_conv3_wgrad_work_bytes(cin, cout, n, h, wd))
    if nb == 0:
        raise ValueError("invalid layer shape")
    work = torch.empty(nb // 4 + 64, dtype=torch.float32, device=g.device)
    dw = torch.empty((cout, 9, cin), dtype=torch.float32, device=g.device)
    db = torch.empty(cout, dtype=torch.float32, device=g.device)
    _check(lib.smg_net_conv3_wgrad(_ptr(g.contiguous()), cout, _ptr(x.contiguous()), cin, _ptr(dw), _ptr(db), n, h, wd,
                                   _ptr(work), ctypes.c_size_t(work.numel() * 4), _stream()))
    return dw, db


def conv3_wgrad_noalloc(g, x, dw=None, db=None):
    """conv3_wgrad through the entry point that allocates nothing (its
    partial sums live in the library's static device array); dw and db may
    be given (float32 (32, 9, c_in) and (32,))."""
    import torch
    n, h, wd, cout = g.shape
    cin = x.shape[3]
    dw = dw if dw is not None else torch.empty((cout, 9, cin), dtype=torch.float32, device=g.device)
    db = db if db is not None else torch.empty(cout, dtype=torch.float32, device=g.device)
    _check(load().smg_net_conv3_wgrad_noalloc(_ptr(g.contiguous()), cout, _ptr(x.contiguous()), cin, _ptr(dw),
                                              _ptr(db), n, h, wd, _stream()))
    return dw, db


def grid_from_spec(spec, **opts):
    """Plan from any object with the GridSpec attributes (geometry, radial,
    n_a, n_b, n_phi, a_min, a_max, b_min, b_max, G)."""
    return Plan(spec.geometry, spec.radial, spec.n_a, spec.n_b, spec.n_phi, spec.a_min, spec.a_max, spec.b_min,
                spec.b_max, spec.G, **opts)


PI = math.pi
