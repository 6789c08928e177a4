"""Thin ctypes binding of the C ABI in include/wdg.h.

Only argument marshalling happens here: every step of the method runs in the
HIP library.  Functions keep the C names; ``Simulation`` bundles the calls a
typical run needs and lets PyTorch own the three device state buffers.

Importing this module loads ``libwdg.so`` from the package directory and raises
ImportError if it has not been built (``python -m paper_2006_02551_amd.build``).

PyTorch ships its own copy of the HIP runtime.  Two HIP runtimes in one
process do not share devices, so torch is imported first: the library's
dependency on libamdhip64.so.7 then resolves to the runtime torch already
loaded, and device pointers and streams from torch are valid in the library.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

try:  # load torch's HIP runtime before the library (see above)
    import torch  # noqa: F401
except ImportError:  # host-only use without torch
    torch = None

HERE = os.path.dirname(os.path.abspath(__file__))
# WDG_LIBRARY selects another build of the same library (the host-sanitizer build of build.py --sanitize)
LIB_PATH = os.environ.get("WDG_LIBRARY") or os.path.join(HERE, "libwdg.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2006_02551_amd.build`")
_lib = C.CDLL(LIB_PATH)

WDG_OK, WDG_EINVAL, WDG_EMESH, WDG_ENOMEM, WDG_EHIP, WDG_ESTATE, WDG_EPROBE, WDG_ENONFINITE = 0, -1, -2, -3, -4, -5, -6, -7
WDG_FP64, WDG_FP32 = 0, 1
WDG_HOST_ONLY = 1
WDG_ALIGN_COMPONENTS = 2
WDG_OP_DR, WDG_OP_DS, WDG_OP_DT, WDG_OP_LIFT, WDG_OP_VQ, WDG_OP_PQ, WDG_OP_M = range(7)
WDG_KERNEL_AUTO, WDG_KERNEL_SCALAR, WDG_KERNEL_MFMA = 0, 1, 2
WDG_SCHEDULE_FORWARD, WDG_SCHEDULE_REVERSED, WDG_SCHEDULE_ALTERNATING = 0, 1, 2
WDG_PML_WAA, WDG_PML_DIRECT, WDG_PML_CONSTANT = 0, 1, 2

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class wdg_mesh(C.Structure):
    _fields_ = [("nv", C.c_int32), ("vxyz", _dp), ("K", C.c_int32), ("etov", _ip), ("vertex_id", _ip)]


class wdg_method(C.Structure):
    _fields_ = [("N", C.c_int32), ("nq", C.c_int32), ("cub_rst", _dp), ("cub_w", _dp),
                ("flux_alpha", C.c_double), ("precision", C.c_int32), ("flags", C.c_int32),
                ("pml_lo", C.c_double * 3), ("pml_hi", C.c_double * 3), ("pml_L", C.c_double * 3),
                ("sigma_max", C.c_double * 3), ("profile_order", C.c_double), ("kappa_max", C.c_double)]


class wdg_dims_t(C.Structure):
    _fields_ = [("K", C.c_int32), ("K_pml", C.c_int32), ("N", C.c_int32), ("Np", C.c_int32),
                ("Nfp", C.c_int32), ("Nq", C.c_int32), ("block", C.c_int32), ("nblk_pml", C.c_int32),
                ("nblk", C.c_int32), ("precision", C.c_int32), ("has_kappa", C.c_int32),
                ("state_bytes", C.c_int64), ("dt_unit", C.c_double), ("time", C.c_double), ("steps", C.c_int64),
                ("kernel", C.c_int32), ("tiles", C.c_int32), ("pml_scheme", C.c_int32)]


class wdg_dipole(C.Structure):
    _fields_ = [("amplitude", C.c_double), ("f0", C.c_double), ("t0", C.c_double), ("tau", C.c_double),
                ("center", C.c_double * 3), ("width", C.c_double), ("direction", C.c_double * 3)]


class wdg_mem_t(C.Structure):
    _fields_ = [("state", C.c_int64), ("geometry", C.c_int64), ("connectivity", C.c_int64),
                ("coefficients", C.c_int64), ("operators", C.c_int64), ("paper_direct", C.c_int64),
                ("paper_waa", C.c_int64), ("scheme_data", C.c_int64)]


_ctx = C.c_void_p


class wdg_shell(C.Structure):
    _fields_ = [("outer_lo", C.c_double * 3), ("outer_hi", C.c_double * 3),
                ("inner_lo", C.c_double * 3), ("inner_hi", C.c_double * 3)]


def _sig(name, res, *args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


wdg_version = _sig("wdg_version", C.c_int32)
wdg_error_string = _sig("wdg_error_string", C.c_char_p, C.c_int32)
wdg_last_error = _sig("wdg_last_error", C.c_char_p, _ctx)
wdg_create = _sig("wdg_create", C.c_int32, C.POINTER(wdg_mesh), C.POINTER(wdg_method), C.POINTER(_ctx))
wdg_destroy = _sig("wdg_destroy", None, _ctx)
wdg_get_dims = _sig("wdg_get_dims", C.c_int32, _ctx, C.POINTER(wdg_dims_t))
wdg_bind_state = _sig("wdg_bind_state", C.c_int32, _ctx, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64)
wdg_set_fields = _sig("wdg_set_fields", C.c_int32, _ctx, _dp)
wdg_get_fields = _sig("wdg_get_fields", C.c_int32, _ctx, _dp)
wdg_get_residual = _sig("wdg_get_residual", C.c_int32, _ctx, _dp)
wdg_set_time = _sig("wdg_set_time", C.c_int32, _ctx, C.c_double)
wdg_set_dipole = _sig("wdg_set_dipole", C.c_int32, _ctx, C.POINTER(wdg_dipole))
wdg_set_probes = _sig("wdg_set_probes", C.c_int32, _ctx, C.c_int32, _dp, C.c_int32)
wdg_probe_read = _sig("wdg_probe_read", C.c_int32, _ctx, _dp, C.c_int32, _ip)
wdg_set_kernel = _sig("wdg_set_kernel", C.c_int32, _ctx, C.c_int32)
wdg_set_pml_scheme = _sig("wdg_set_pml_scheme", C.c_int32, _ctx, C.c_int32, C.c_int32, _dp, _dp)
wdg_step = _sig("wdg_step", C.c_int32, _ctx, C.c_double, C.c_int32, C.c_void_p)
wdg_rhs = _sig("wdg_rhs", C.c_int32, _ctx, C.c_double, C.c_void_p)
wdg_energy = _sig("wdg_energy", C.c_int32, _ctx, _dp, C.c_void_p)
wdg_node_coords = _sig("wdg_node_coords", C.c_int32, _ctx, _dp)
wdg_reference_op = _sig("wdg_reference_op", C.c_int32, _ctx, C.c_int32, _dp)
wdg_element_info = _sig("wdg_element_info", C.c_int32, _ctx, _dp, _dp, _dp, _ip, _ip, _ip)
wdg_memory_report = _sig("wdg_memory_report", C.c_int32, _ctx, C.POINTER(wdg_mem_t))
wdg_set_tiles = _sig("wdg_set_tiles", C.c_int32, _ctx, C.c_int32)
wdg_set_waa_shortcut = _sig("wdg_set_waa_shortcut", C.c_int32, _ctx, C.c_int32)
wdg_set_schedule = _sig("wdg_set_schedule", C.c_int32, _ctx, C.c_int32)
wdg_element_slots = _sig("wdg_element_slots", C.c_int32, _ctx, C.POINTER(C.c_int32))
wdg_set_step_groups = _sig("wdg_set_step_groups", C.c_int32, _ctx, C.c_int32, C.POINTER(C.c_int32))
wdg_autotune_cached = _sig("wdg_autotune_cached", C.c_int32, _ctx, C.c_int32, C.c_void_p, C.POINTER(C.c_int32))
wdg_energy_noalloc = _sig("wdg_energy_noalloc", C.c_int32, _ctx, C.c_void_p, C.c_void_p)
wdg_measure_copy_bandwidth = _sig("wdg_measure_copy_bandwidth", C.c_int32, C.c_int64, C.c_void_p, _dp)
wdg_measure_mfma_peak = _sig("wdg_measure_mfma_peak", C.c_int32, C.c_int32, C.c_int32, C.c_void_p, _dp)
wdg_autotune = _sig("wdg_autotune", C.c_int32, _ctx, C.c_int32, _dp, C.c_void_p)
wdg_step_graph = _sig("wdg_step_graph", C.c_int32, _ctx, C.c_double, C.c_int32, C.c_void_p)
wdg_set_dt_scale = _sig("wdg_set_dt_scale", C.c_int32, _ctx, _dp)
wdg_set_sigma_profile = _sig("wdg_set_sigma_profile", C.c_int32, _ctx, _ip, C.c_int32, _dp, _dp)
wdg_set_sigma_q = _sig("wdg_set_sigma_q", C.c_int32, _ctx, _dp)
wdg_get_sigma_q = _sig("wdg_get_sigma_q", C.c_int32, _ctx, _dp)
wdg_cubature_points = _sig("wdg_cubature_points", C.c_int32, _ctx, _dp)
wdg_set_pml_profile = _sig("wdg_set_pml_profile", C.c_int32, _ctx, _dp, _dp, C.c_double)
wdg_shell_energy = _sig("wdg_shell_energy", C.c_int32, _ctx, C.POINTER(wdg_shell), _dp, C.c_void_p)
wdg_loss_gradient = _sig("wdg_loss_gradient", C.c_int32, _ctx, C.c_double, C.c_int32, C.POINTER(wdg_shell), C.c_int32,
                         _dp, _dp, _dp, C.c_void_p)


class WdgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


def _check(rc, ctx=None):
    if rc != WDG_OK:
        msg = wdg_last_error(ctx)
        raise WdgError(rc, (msg or wdg_error_string(rc)).decode() if isinstance(msg, bytes) else str(msg))
    return rc


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, t=_dp):
    return a.ctypes.data_as(t)


def make_method(N, rule, pml, alpha=1.0, precision=WDG_FP64, flags=0):
    """Fill a wdg_method; keeps references to the arrays it points into."""
    rst, w = _f64(rule[0]), _f64(rule[1])
    m = wdg_method()
    m.N = int(N)
    m.nq = len(w)
    m.cub_rst = _ptr(rst)
    m.cub_w = _ptr(w)
    m.flux_alpha = float(alpha)
    m.precision = int(precision)
    m.flags = int(flags)
    pml = pml or {"lo": [-1e30] * 3, "hi": [1e30] * 3, "L": [1.0] * 3, "sigma_max": [0.0] * 3,
                  "order": 1.0, "kappa_max": 1.0}
    for i in range(3):
        m.pml_lo[i] = float(pml["lo"][i])
        m.pml_hi[i] = float(pml["hi"][i])
        m.pml_L[i] = float(pml["L"][i])
        m.sigma_max[i] = float(pml["sigma_max"][i])
    m.profile_order = float(pml["order"])
    m.kappa_max = float(pml.get("kappa_max", 1.0))
    m._keep = (rst, w)
    return m


def make_mesh(vxyz, etov, vertex_id=None):
    v = _f64(vxyz)
    e = np.ascontiguousarray(etov, dtype=np.int32)
    m = wdg_mesh()
    m.nv = v.shape[0]
    m.vxyz = _ptr(v)
    m.K = e.shape[0]
    m.etov = _ptr(e, _ip)
    vid = None
    if vertex_id is not None:
        vid = np.ascontiguousarray(vertex_id, dtype=np.int32)
        assert vid.shape == (v.shape[0],)
        m.vertex_id = _ptr(vid, _ip)
    m._keep = (v, e, vid)
    return m


class Context:
    """Owns a wdg_ctx; host-only contexts need no GPU."""

    def __init__(self, vxyz, etov, N, rule, pml, alpha=1.0, precision=WDG_FP64, host_only=False, vertex_id=None,
                 flags=0):
        mesh = make_mesh(vxyz, etov, vertex_id)
        meth = make_method(N, rule, pml, alpha, precision, (WDG_HOST_ONLY if host_only else 0) | int(flags))
        h = _ctx()
        _check(wdg_create(C.byref(mesh), C.byref(meth), C.byref(h)))
        self.h = h
        self.dims = self.get_dims()

    def __del__(self):
        h = getattr(self, "h", None)
        if h and wdg_destroy is not None:
            wdg_destroy(h)
            self.h = None

    def element_slots(self):
        """Device slot (block * 64 + lane) of every element, [K] int32."""
        out = np.zeros(self.dims.K, dtype=np.int32)
        _check(wdg_element_slots(self.h, out.ctypes.data_as(C.POINTER(C.c_int32))), self.h)
        return out

    def get_dims(self):
        d = wdg_dims_t()
        _check(wdg_get_dims(self.h, C.byref(d)), self.h)
        return d

    def node_coords(self):
        d = self.dims
        out = np.zeros((d.K, d.Np, 3))
        _check(wdg_node_coords(self.h, _ptr(out)), self.h)
        return out

    def reference_op(self, which):
        d = self.dims
        shape = {WDG_OP_DR: (d.Np, d.Np), WDG_OP_DS: (d.Np, d.Np), WDG_OP_DT: (d.Np, d.Np),
                 WDG_OP_LIFT: (d.Np, 4 * d.Nfp), WDG_OP_VQ: (d.Nq, d.Np), WDG_OP_PQ: (d.Np, d.Nq),
                 WDG_OP_M: (d.Np, d.Np)}[which]
        out = np.zeros(shape)
        _check(wdg_reference_op(self.h, which, _ptr(out)), self.h)
        return out

    def element_info(self):
        K = self.dims.K
        J, Fs, nrm = np.zeros(K), np.zeros((K, 4)), np.zeros((K, 4, 3))
        etoe, etof, ispml = (np.zeros((K, 4), np.int32), np.zeros((K, 4), np.int32), np.zeros(K, np.int32))
        _check(wdg_element_info(self.h, _ptr(J), _ptr(Fs), _ptr(nrm), _ptr(etoe, _ip), _ptr(etof, _ip),
                                _ptr(ispml, _ip)), self.h)
        return {"J": J, "Fscale": Fs, "normals": nrm, "etoe": etoe, "etof": etof, "is_pml": ispml.astype(bool)}

    def memory_report(self):
        m = wdg_mem_t()
        _check(wdg_memory_report(self.h, C.byref(m)), self.h)
        return {k: getattr(m, k) for k, _ in wdg_mem_t._fields_}

    def cubature_points(self):
        d = self.dims
        out = np.zeros((d.K, d.Nq, 3))
        _check(wdg_cubature_points(self.h, _ptr(out)), self.h)
        return out

    def set_sigma_profile(self, group, sigma_max, order):
        """Per-group profiles: group [K] int, sigma_max [G, 3], order [G]."""
        g = np.ascontiguousarray(group, dtype=np.int32)
        sm = _f64(np.asarray(sigma_max, dtype=np.float64).reshape(-1, 3))
        od = _f64(np.asarray(order, dtype=np.float64).reshape(-1))
        assert g.shape == (self.dims.K,) and len(sm) == len(od)
        _check(wdg_set_sigma_profile(self.h, _ptr(g, _ip), len(od), _ptr(sm), _ptr(od)), self.h)

    def get_sigma_q(self):
        d = self.dims
        out = np.zeros((d.K, d.Nq, 3))
        _check(wdg_get_sigma_q(self.h, _ptr(out)), self.h)
        return out

    def set_pml_profile(self, sigma_max, L, order):
        """Re-samples sigma at the cubature points from the layer profile with new (sigma_max [3], L [3], order)."""
        sm = _f64(np.broadcast_to(np.asarray(sigma_max, dtype=np.float64), (3,)))
        ll = _f64(np.broadcast_to(np.asarray(L, dtype=np.float64), (3,)))
        _check(wdg_set_pml_profile(self.h, _ptr(sm), _ptr(ll), float(order)), self.h)

    def set_sigma_q(self, sigma):
        sigma = _f64(sigma)
        d = self.dims
        assert sigma.shape == (d.K, d.Nq, 3)
        _check(wdg_set_sigma_q(self.h, _ptr(sigma)), self.h)


class Simulation(Context):
    """A device context whose three state buffers are PyTorch CUDA (HIP) tensors."""

    def __init__(self, vxyz, etov, N, rule, pml, alpha=1.0, precision=WDG_FP64, device="cuda", vertex_id=None,
                 flags=0):
        super().__init__(vxyz, etov, N, rule, pml, alpha, precision, host_only=False, vertex_id=vertex_id, flags=flags)
        nbytes = self.dims.state_bytes
        self.bufs = [torch.empty(nbytes, dtype=torch.uint8, device=device) for _ in range(3)]
        _check(wdg_bind_state(self.h, C.c_void_p(self.bufs[0].data_ptr()), C.c_void_p(self.bufs[1].data_ptr()),
                              C.c_void_p(self.bufs[2].data_ptr()), nbytes), self.h)
        self.nprobe = 0

    @staticmethod
    def _stream(stream):
        if stream is None:
            stream = torch.cuda.current_stream()
        return C.c_void_p(stream.cuda_stream)

    def set_fields(self, q):
        q = _f64(q)
        d = self.dims
        assert q.shape == (d.K, 12, d.Np)
        _check(wdg_set_fields(self.h, _ptr(q)), self.h)

    def get_fields(self):
        d = self.dims
        out = np.zeros((d.K, 12, d.Np))
        _check(wdg_get_fields(self.h, _ptr(out)), self.h)
        return out

    def get_residual(self):
        d = self.dims
        out = np.zeros((d.K, 12, d.Np))
        _check(wdg_get_residual(self.h, _ptr(out)), self.h)
        return out

    def set_time(self, t):
        _check(wdg_set_time(self.h, float(t)), self.h)

    def set_dipole(self, src):
        if src is None:
            _check(wdg_set_dipole(self.h, None), self.h)
            return
        d = wdg_dipole()
        d.amplitude, d.f0, d.t0, d.tau, d.width = (float(src[k]) for k in ("amplitude", "f0", "t0", "tau", "width"))
        for i in range(3):
            d.center[i] = float(src["center"][i])
            d.direction[i] = float(src["direction"][i])
        _check(wdg_set_dipole(self.h, C.byref(d)), self.h)

    def set_probes(self, xyz, capacity):
        xyz = _f64(xyz).reshape(-1, 3)
        _check(wdg_set_probes(self.h, len(xyz), _ptr(xyz), int(capacity)), self.h)
        self.nprobe = len(xyz)

    def probe_read(self, max_rows):
        out = np.zeros((max(int(max_rows), 1), max(self.nprobe, 1), 6))
        n = C.c_int32(0)
        _check(wdg_probe_read(self.h, _ptr(out), int(max_rows), C.byref(n)), self.h)
        return out[:n.value, :self.nprobe]

    def set_kernel(self, variant):
        _check(wdg_set_kernel(self.h, int(variant)), self.h)
        self.dims = self.get_dims()

    def set_pml_scheme(self, scheme, rule=None):
        """WDG_PML_WAA, WDG_PML_DIRECT (rule = (rst [nr, 3], w [nr]) for the weighted mass matrices) or
        WDG_PML_CONSTANT."""
        if rule is None:
            _check(wdg_set_pml_scheme(self.h, int(scheme), 0, None, None), self.h)
        else:
            rst, w = _f64(np.asarray(rule[0]).reshape(-1, 3)), _f64(np.asarray(rule[1]).reshape(-1))
            assert len(rst) == len(w)
            _check(wdg_set_pml_scheme(self.h, int(scheme), len(w), _ptr(rst), _ptr(w)), self.h)
        self.dims = self.get_dims()

    def step(self, dt, nsteps, stream=None):
        _check(wdg_step(self.h, float(dt), int(nsteps), self._stream(stream)), self.h)

    def step_graph(self, dt, nsteps, stream=None):
        """Like step, replaying a captured two-step HIP graph (needs a non-default stream)."""
        _check(wdg_step_graph(self.h, float(dt), int(nsteps), self._stream(stream)), self.h)

    def set_tiles(self, tiles):
        _check(wdg_set_tiles(self.h, int(tiles)), self.h)
        self.dims = self.get_dims()

    def set_step_groups(self, group, ngroups=None):
        """Groups of independent simulations for captured stepping (group [K] int, or None to remove)."""
        if group is None:
            _check(wdg_set_step_groups(self.h, 0, None), self.h)
            return
        g = np.ascontiguousarray(group, dtype=np.int32)
        n = int(g.max()) + 1 if ngroups is None else int(ngroups)
        _check(wdg_set_step_groups(self.h, n, g.ctypes.data_as(C.POINTER(C.c_int32))), self.h)

    def set_schedule(self, mode):
        """WDG_SCHEDULE_FORWARD, WDG_SCHEDULE_REVERSED or WDG_SCHEDULE_ALTERNATING (the default)."""
        _check(wdg_set_schedule(self.h, int(mode)), self.h)

    def set_waa_shortcut(self, on):
        """Skip (True) or apply (False, the default) the weight-adjusted inverse where it is the identity."""
        _check(wdg_set_waa_shortcut(self.h, int(bool(on))), self.h)

    def autotune_cached(self, reps=5, stream=None):
        """Applies the cached stage-kernel choice for this kind of context, or times and caches one;
        returns True when the choice came from the cache."""
        hit = C.c_int32(0)
        _check(wdg_autotune_cached(self.h, int(reps), self._stream(stream), C.byref(hit)), self.h)
        self.dims = self.get_dims()
        return bool(hit.value)

    def autotune(self, reps=5, stream=None):
        """Times the stage kernels and keeps the fastest; returns us per launch
        {'scalar': t, 'mfma_1tile': t, 'mfma_2tiles': t} (None where unavailable)."""
        t = np.zeros(3)
        _check(wdg_autotune(self.h, int(reps), _ptr(t), self._stream(stream)), self.h)
        self.dims = self.get_dims()
        return {k: (None if v < 0 else float(v)) for k, v in zip(("scalar", "mfma_1tile", "mfma_2tiles"), t)}

    def set_dt_scale(self, scale):
        if scale is None:
            _check(wdg_set_dt_scale(self.h, None), self.h)
            return
        sc = _f64(np.asarray(scale, dtype=np.float64).reshape(-1))
        assert sc.shape == (self.dims.K,)
        _check(wdg_set_dt_scale(self.h, _ptr(sc)), self.h)

    def rhs(self, t, stream=None):
        _check(wdg_rhs(self.h, float(t), self._stream(stream)), self.h)

    def energy(self, stream=None):
        e = C.c_double(0.0)
        _check(wdg_energy(self.h, C.byref(e), self._stream(stream)), self.h)
        return e.value

    def shell_energy(self, shell, stream=None):
        e = C.c_double(0.0)
        sh = make_shell(shell)
        _check(wdg_shell_energy(self.h, C.byref(sh), C.byref(e), self._stream(stream)), self.h)
        return e.value

    def loss_gradient(self, dt, nsteps, shell, checkpoint_interval=0, stream=None, profile=True):
        """(J, dJ/dsigma [K, Nq, 3], dJ/d(sigma_max xyz, L xyz, order) [7] or None when profile is False);
        the state advances nsteps steps."""
        d = self.dims
        loss = C.c_double(0.0)
        gs = np.zeros((d.K, d.Nq, 3))
        gp = np.zeros(7) if profile else None
        sh = make_shell(shell)
        _check(wdg_loss_gradient(self.h, float(dt), int(nsteps), C.byref(sh), int(checkpoint_interval), C.byref(loss),
                                 _ptr(gs), _ptr(gp) if profile else None, self._stream(stream)), self.h)
        return loss.value, gs, gp


def measure_mfma_peak(precision, iters=4000, stream=None):
    """Sustained TFLOP/s of the 16x16x4 MFMA of the given precision on the current device."""
    out = C.c_double(0.0)
    st = None if stream is None else C.c_void_p(stream.cuda_stream)
    rc = wdg_measure_mfma_peak(int(precision), int(iters), st, C.byref(out))
    if rc != WDG_OK:
        raise WdgError(rc, f"wdg_measure_mfma_peak failed ({rc})")
    return out.value


def measure_copy_bandwidth(nbytes=1 << 30, stream=None):
    """GB/s (read + written) of the library's plain device copy of nbytes bytes."""
    out = C.c_double(0.0)
    st = None if stream is None else C.c_void_p(stream.cuda_stream)
    rc = wdg_measure_copy_bandwidth(int(nbytes), st, C.byref(out))
    if rc != WDG_OK:
        raise WdgError(rc, f"wdg_measure_copy_bandwidth failed ({rc})")
    return out.value


def make_shell(shell) -> wdg_shell:
    sh = wdg_shell()
    for i in range(3):
        sh.outer_lo[i], sh.outer_hi[i] = float(shell["outer_lo"][i]), float(shell["outer_hi"][i])
        sh.inner_lo[i], sh.inner_hi[i] = float(shell["inner_lo"][i]), float(shell["inner_hi"][i])
    return sh


class ShellLoss(torch.autograd.Function):
    """Loss sum_{n=1..nsteps} dt E_shell(q_n) as a function of sigma at the cubature points.

    forward(sigma_q [K, Nq, 3] float64 tensor, sim, q0, t0, dt, nsteps, shell, checkpoint_interval) sets sigma,
    the fields q0 and the time t0 on `sim`, runs the library's loss and adjoint sweep once and keeps
    dJ/dsigma for backward."""

    @staticmethod
    def forward(ctx, sigma_q, sim, q0, t0, dt, nsteps, shell, checkpoint_interval=0):
        sim.set_sigma_q(sigma_q.detach().cpu().numpy())
        sim.set_fields(q0)
        sim.set_time(t0)
        loss, gs, _ = sim.loss_gradient(dt, nsteps, shell, checkpoint_interval, profile=False)
        ctx.save_for_backward(torch.from_numpy(gs).to(sigma_q.device, sigma_q.dtype))
        return torch.tensor(loss, dtype=sigma_q.dtype, device=sigma_q.device)

    @staticmethod
    def backward(ctx, gout):
        (g,) = ctx.saved_tensors
        return (gout * g, None, None, None, None, None, None, None)


class ProfileLoss(torch.autograd.Function):
    """Loss sum_{n=1..nsteps} dt E_shell(q_n) as a function of the layer profile theta = (sigma_max x,y,z,
    L x,y,z, order), a float64 tensor [7].

    forward(theta, sim, q0, t0, dt, nsteps, shell, checkpoint_interval) re-samples sigma on `sim` from theta
    (outer wall fixed, the interface moving with L), sets the fields q0 and the time t0, runs the library's
    loss and adjoint sweep once and keeps the library's dJ/dtheta for backward."""

    @staticmethod
    def forward(ctx, theta, sim, q0, t0, dt, nsteps, shell, checkpoint_interval=0):
        th = theta.detach().cpu().numpy().astype(np.float64)
        sim.set_pml_profile(th[0:3], th[3:6], th[6])
        sim.set_fields(q0)
        sim.set_time(t0)
        loss, _, gp = sim.loss_gradient(dt, nsteps, shell, checkpoint_interval)
        ctx.save_for_backward(torch.from_numpy(gp).to(theta.device, theta.dtype))
        return torch.tensor(loss, dtype=theta.dtype, device=theta.device)

    @staticmethod
    def backward(ctx, gout):
        (g,) = ctx.saved_tensors
        return (gout * g, None, None, None, None, None, None, None)
