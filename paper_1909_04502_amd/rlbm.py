"""ctypes binding of the RLBM C ABI (``include/rlbm.h``).

Argument marshalling only: every step of the update runs in the HIP kernels of
``librlbm.so``.  PyTorch provides device memory and the current stream; the
library is loaded after torch so that both use the same HIP runtime.  A
missing library is an error (there is no fallback path).
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, Structure, c_char_p, c_double, c_int32, c_int64, c_void_p

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librlbm.so")

OK, ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_QUADRATURE, ERR_DEVICE, ERR_NONPHYSICAL = range(6)
KIND = {"ur_onlattice": 0, "product": 1, "massive_onlattice": 2}
STORAGE = {"f64": 0, "f32dev": 1, "f32dev_f64": 2}
BC = {"periodic": 0, "open": 1, "wall": 2}


class Model(Structure):
    _fields_ = [("d", c_int32), ("order", c_int32), ("kind", c_int32), ("pad_", c_int32), ("zeta", c_double),
                ("v0", c_double)]


class Config(Structure):
    _fields_ = [("model", Model), ("extent", c_int64 * 3), ("bc", c_int32 * 3), ("storage", c_int32),
                ("tau", c_double), ("tau_field", c_void_p), ("n_ref", c_double), ("force", c_double * 3),
                ("tau_T", c_double), ("wall_T", (c_double * 2) * 3)]


class Info(Structure):
    _fields_ = [("Q", c_int32), ("n_basis", c_int32), ("sites", c_int64), ("state_bytes", c_int64),
                ("elem_bytes", c_int32), ("on_lattice", c_int32), ("v0", c_double)]


class Fields(Structure):
    _fields_ = [("n", c_void_p), ("eps", c_void_p), ("T", c_void_p), ("U", c_void_p)]


class RLBMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"rlbm status {status}: {msg}")
        self.status = status


_lib = None


def _check_single_hip_runtime():
    """Refuse to run with two HIP runtimes mapped (ours and torch's must be the same object)."""
    paths = set()
    try:
        with open("/proc/self/maps") as fh:
            for line in fh:
                if "libamdhip64" in line:
                    paths.add(os.path.realpath(line.split()[-1]))
    except OSError:
        return
    if len(paths) > 1:
        raise RuntimeError("two HIP runtimes are loaded: " + ", ".join(sorted(paths)))


def lib():
    """Load librlbm.so (built in place by paper_1909_04502_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run paper_1909_04502_amd.build.build()")
    L = ctypes.CDLL(LIB_PATH)
    st = c_int32
    L.rlbm_status_string.restype = c_char_p
    L.rlbm_status_string.argtypes = [st]
    L.rlbm_last_error.restype = c_char_p
    L.rlbm_last_error.argtypes = []
    L.rlbm_quadrature_build.restype = st
    L.rlbm_quadrature_build.argtypes = [POINTER(Model), POINTER(c_int32), c_void_p, c_void_p, c_void_p]
    L.rlbm_massive_window.restype = st
    L.rlbm_massive_window.argtypes = [POINTER(Model), POINTER(c_double), POINTER(c_double)]
    L.rlbm_create.restype = st
    L.rlbm_create.argtypes = [POINTER(Config), POINTER(c_void_p)]
    L.rlbm_destroy.restype = st
    L.rlbm_destroy.argtypes = [c_void_p]
    L.rlbm_get_info.restype = st
    L.rlbm_get_info.argtypes = [c_void_p, POINTER(Info)]
    L.rlbm_init.restype = st
    L.rlbm_init.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_void_p,
                            POINTER(Fields), c_void_p]
    L.rlbm_step.restype = st
    L.rlbm_step.argtypes = [c_void_p, c_void_p, c_void_p, c_int32, POINTER(Fields), c_void_p]
    L.rlbm_step_static.restype = st
    L.rlbm_step_static.argtypes = [POINTER(Config), c_void_p, c_void_p, c_int32, POINTER(Fields), c_void_p,
                                   c_void_p]
    L.rlbm_moments.restype = st
    L.rlbm_moments.argtypes = [c_void_p, c_void_p, POINTER(Fields), c_void_p]
    L.rlbm_sync.restype = st
    L.rlbm_sync.argtypes = [c_void_p, c_void_p]
    L.rlbm_adjoint_step.restype = st
    L.rlbm_adjoint_step.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
    L.rlbm_moments_vjp.restype = st
    L.rlbm_moments_vjp.argtypes = [c_void_p, c_void_p, POINTER(Fields), c_void_p, c_void_p]
    L.rlbm_init_vjp.restype = st
    L.rlbm_init_vjp.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_void_p,
                                c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
    L.rlbm_variant_count.restype = c_int32
    L.rlbm_variant_count.argtypes = []
    L.rlbm_set_variant.restype = st
    L.rlbm_set_variant.argtypes = [c_void_p, c_int32]
    L.rlbm_get_variant.restype = st
    L.rlbm_get_variant.argtypes = [c_void_p, POINTER(c_int32)]
    L.rlbm_set_store_mode.restype = st
    L.rlbm_set_store_mode.argtypes = [c_void_p, c_int32]
    L.rlbm_get_store_mode.restype = st
    L.rlbm_get_store_mode.argtypes = [c_void_p, POINTER(c_int32), POINTER(c_int32)]
    L.rlbm_autotune.restype = st
    L.rlbm_autotune.argtypes = [c_void_p, c_int32, c_void_p, c_void_p]
    L.rlbm_batch_create.restype = st
    L.rlbm_batch_create.argtypes = [POINTER(Config), c_int32, POINTER(c_void_p)]
    L.rlbm_batch_destroy.restype = st
    L.rlbm_batch_destroy.argtypes = [c_void_p]
    L.rlbm_batch_layout.restype = st
    L.rlbm_batch_layout.argtypes = [c_void_p, POINTER(c_int64), POINTER(c_int64), c_void_p, c_void_p]
    L.rlbm_batch_lattice.restype = st
    L.rlbm_batch_lattice.argtypes = [c_void_p, c_int32, POINTER(c_void_p)]
    L.rlbm_batch_init.restype = st
    L.rlbm_batch_init.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
    L.rlbm_batch_step.restype = st
    L.rlbm_batch_step.argtypes = [c_void_p, c_void_p, c_void_p, c_int32, c_int32, c_void_p]
    L.rlbm_batch_moments.restype = st
    L.rlbm_batch_moments.argtypes = [c_void_p, c_void_p, POINTER(Fields), c_void_p]
    L.rlbm_batch_sync.restype = st
    L.rlbm_batch_sync.argtypes = [c_void_p, c_void_p]
    L.rlbm_batch_variant_count.restype = c_int32
    L.rlbm_batch_variant_count.argtypes = []
    L.rlbm_batch_set_variant.restype = st
    L.rlbm_batch_set_variant.argtypes = [c_void_p, c_int32]
    L.rlbm_batch_get_variant.restype = st
    L.rlbm_batch_get_variant.argtypes = [c_void_p, POINTER(c_int32)]
    L.rlbm_batch_set_store_mode.restype = st
    L.rlbm_batch_set_store_mode.argtypes = [c_void_p, c_int32]
    L.rlbm_batch_get_store_mode.restype = st
    L.rlbm_batch_get_store_mode.argtypes = [c_void_p, POINTER(c_int32), POINTER(c_int32)]
    L.rlbm_batch_autotune.restype = st
    L.rlbm_batch_autotune.argtypes = [c_void_p, c_void_p, c_void_p, c_int32, c_void_p, c_void_p]
    L.rlbm_copy_planes.restype = st
    L.rlbm_copy_planes.argtypes = [c_void_p, c_void_p, c_int64, c_int32, c_int32, c_int32, c_int32, c_void_p]
    _lib = L
    _check_single_hip_runtime()
    return L


def _check(status):
    if status != OK:
        L = lib()
        raise RLBMError(status, L.rlbm_last_error().decode() or L.rlbm_status_string(status).decode())


def _model(d, zeta, order, kind, v0=0.0):
    return Model(d=d, order=order, kind=KIND[kind] if isinstance(kind, str) else int(kind), pad_=0, zeta=float(zeta),
                 v0=float(v0))


def quadrature_build(d: int, zeta: float, order: int, kind="product", v0=0.0):
    """Host-side quadrature of the library: (p [Q, d+1], w [Q], disp [Q, d]) as float64 CPU tensors.
    v0: massive on-lattice rules only (0 = the middle of the window of non-negative weights)."""
    L = lib()
    m = _model(d, zeta, order, kind, v0)
    Q = c_int32(0)
    _check(L.rlbm_quadrature_build(ctypes.byref(m), ctypes.byref(Q), None, None, None))
    p = torch.empty((Q.value, d + 1), dtype=torch.float64)
    w = torch.empty((Q.value,), dtype=torch.float64)
    disp = torch.empty((Q.value, d), dtype=torch.float64)
    _check(L.rlbm_quadrature_build(ctypes.byref(m), ctypes.byref(Q), p.data_ptr(), w.data_ptr(), disp.data_ptr()))
    return p, w, disp


def massive_window(zeta: float, order: int, d: int = 2):
    """(lo, hi): the v0 interval of non-negative weights of the massive on-lattice rule (Sec. 5.3)."""
    L = lib()
    m = _model(d, zeta, order, "massive_onlattice")
    lo, hi = c_double(0.0), c_double(0.0)
    _check(L.rlbm_massive_window(ctypes.byref(m), ctypes.byref(lo), ctypes.byref(hi)))
    return lo.value, hi.value


def copy_planes(src, dst, planes: int, mode: str = "site", nontemporal: bool = False):
    """dst <- src with rlbm_copy_planes: "site" copies `planes` SoA planes one site per thread (the
    step kernels' access pattern), "flat" as 16-byte vectors.  Both tensors on the device, same size."""
    assert src.is_cuda and dst.is_cuda and src.numel() == dst.numel() and src.dtype == dst.dtype
    es = src.element_size()
    sites = src.numel() // planes
    _check(lib().rlbm_copy_planes(_ptr(src), _ptr(dst), int(sites), int(planes), int(es),
                                  {"site": 0, "flat": 1}[mode], int(bool(nontemporal)), _stream()))


def _stream():
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else c_void_p(t.data_ptr())


class Lattice:
    """One lattice: handle of the C ABI plus the torch-side shapes."""

    def __init__(self, d=2, zeta=1.0, order=3, kind="product", extent=(64, 64), bc=None, storage="f64",
                 tau=0.8, tau_field=None, n_ref=1.0, force=None, v0=0.0, tau_T=0.0, wall_T=None,
                 _handle=None):
        L = lib()
        self._owned = _handle is None
        self.d = d
        self.extent = tuple(int(e) for e in extent)
        if bc is None:
            bc = ("periodic",) * d
        self.storage = storage
        self.dtype = torch.float64 if storage == "f64" else torch.float32
        self.grid_shape = tuple(reversed(self.extent))
        if tau_field is not None:
            tau_field = tau_field.to(device="cuda", dtype=self.dtype).contiguous()
            assert tuple(tau_field.shape) == self.grid_shape
        self.tau_field = tau_field          # kept alive: the handle stores its pointer
        cfg = Config()
        cfg.model = _model(d, zeta, order, kind, v0)
        ext = list(self.extent) + [1] * (3 - d)
        for a in range(3):
            cfg.extent[a] = ext[a]
            cfg.bc[a] = BC[bc[a]] if a < d else 0
        cfg.storage = STORAGE[storage]
        cfg.tau = float(tau)
        cfg.tau_field = tau_field.data_ptr() if tau_field is not None else None
        cfg.n_ref = float(n_ref)
        cfg.tau_T = float(tau_T)
        if wall_T is not None:          # per axis (first plane, last plane); 0 = own temperature
            for a, pair in enumerate(wall_T):
                cfg.wall_T[a][0], cfg.wall_T[a][1] = float(pair[0]), float(pair[1])
        self.force = tuple(float(g) for g in force) if force is not None else (0.0,) * d
        for a in range(3):
            cfg.force[a] = self.force[a] if a < len(self.force) else 0.0
        self.cfg = cfg
        if _handle is None:
            h = c_void_p()
            _check(L.rlbm_create(ctypes.byref(cfg), ctypes.byref(h)))
        else:
            h = _handle                     # a member of a batch: the batch owns it
        self.h = h
        info = Info()
        _check(L.rlbm_get_info(h, ctypes.byref(info)))
        self.Q = info.Q
        self.n_basis = info.n_basis
        self.sites = info.sites
        self.on_lattice = bool(info.on_lattice)
        self.v0 = info.v0

    def __del__(self):
        h = getattr(self, "h", None)
        if getattr(self, "_owned", False) and h is not None and h.value is not None and _lib is not None:
            _lib.rlbm_destroy(h)
        self.h = None

    # ------------------------------------------------------------------
    def new_state(self):
        return torch.empty((self.Q,) + self.grid_shape, dtype=self.dtype, device="cuda")

    def new_fields(self):
        g = self.grid_shape
        dev = "cuda"
        return {"n": torch.empty(g, dtype=torch.float64, device=dev),
                "eps": torch.empty(g, dtype=torch.float64, device=dev),
                "T": torch.empty(g, dtype=torch.float64, device=dev),
                "U": torch.empty((self.d + 1,) + g, dtype=torch.float64, device=dev)}

    @staticmethod
    def _fields_struct(fd):
        if fd is None:
            return None
        return Fields(n=fd["n"].data_ptr(), eps=fd["eps"].data_ptr(), T=fd["T"].data_ptr(), U=fd["U"].data_ptr())

    def _dev64(self, t, shape):
        t = torch.as_tensor(t, dtype=torch.float64).to("cuda").contiguous()
        assert tuple(t.shape) == tuple(shape), (t.shape, shape)
        return t

    def init(self, n0, T0, u0, noise=None, amp=0.0, out=None, want_fields=False):
        """Post-collision state f*(x, 0) from the initial fields (see rlbm_init)."""
        g = self.grid_shape
        n0 = self._dev64(n0, g)
        T0 = self._dev64(T0, g)
        u0 = self._dev64(u0, (self.d,) + g)
        if noise is not None:
            noise = self._dev64(noise, (self.Q,) + g)
        out = self.new_state() if out is None else out
        fd = self.new_fields() if want_fields else None
        fs = self._fields_struct(fd)
        _check(lib().rlbm_init(self.h, _ptr(n0), _ptr(T0), _ptr(u0), _ptr(noise), float(amp), _ptr(out),
                               ctypes.byref(fs) if fs is not None else None, _stream()))
        self._keep = (n0, T0, u0, noise)
        return (out, fd) if want_fields else out

    def step(self, f_a, f_b, nsteps, want_last=False):
        """Advance nsteps; returns the buffer holding the result (and the last fields)."""
        assert f_a.dtype == self.dtype and f_b.dtype == self.dtype
        fd = self.new_fields() if want_last else None
        fs = self._fields_struct(fd)
        _check(lib().rlbm_step(self.h, _ptr(f_a), _ptr(f_b), int(nsteps),
                               ctypes.byref(fs) if fs is not None else None, _stream()))
        res = f_b if nsteps % 2 == 1 else f_a
        return (res, fd) if want_last else res

    def step_static(self, f_a, f_b, nsteps, flag=None):
        """rlbm_step_static on this lattice's configuration (no handle, no device allocation);
        flag: optional device int32 tensor set to 1 on a non-physical state.  Returns the buffer
        holding the result."""
        assert f_a.dtype == self.dtype and f_b.dtype == self.dtype
        _check(lib().rlbm_step_static(ctypes.byref(self.cfg), _ptr(f_a), _ptr(f_b), int(nsteps), None, _ptr(flag),
                                      _stream()))
        return f_b if nsteps % 2 == 1 else f_a

    def moments(self, f):
        """Macroscopic fields of the streamed populations of state f."""
        fd = self.new_fields()
        fs = self._fields_struct(fd)
        _check(lib().rlbm_moments(self.h, _ptr(f), ctypes.byref(fs), _stream()))
        return fd

    def sync(self):
        _check(lib().rlbm_sync(self.h, _stream()))

    # reverse mode --------------------------------------------------------
    def adjoint_step(self, f_prev, lam_next, lam=None, dtau=None):
        """lam_t = J_C(S f_prev)^T S^T lam_next; dtau (double [grid]) accumulates dL/dtau."""
        lam = torch.empty_like(lam_next) if lam is None else lam
        _check(lib().rlbm_adjoint_step(self.h, _ptr(f_prev), _ptr(lam_next), _ptr(lam), _ptr(dtau), _stream()))
        return lam

    def moments_vjp(self, f, gn=None, geps=None, gT=None, gU=None, lam=None):
        """dL/dF of the streamed populations of f given dL/d(n, eps, T, U) (any may be None)."""
        g = self.grid_shape

        def dev(t, shape):
            return None if t is None else self._dev64(t, shape)
        gn, geps, gT = dev(gn, g), dev(geps, g), dev(gT, g)
        gU = dev(gU, (self.d + 1,) + g)
        fs = Fields(n=_ptr(gn), eps=_ptr(geps), T=_ptr(gT), U=_ptr(gU))
        lam = self.new_state() if lam is None else lam
        _check(lib().rlbm_moments_vjp(self.h, _ptr(f), ctypes.byref(fs), _ptr(lam), _stream()))
        self._keep_vjp = (gn, geps, gT, gU)
        return lam

    def init_vjp(self, n0, T0, u0, lam1, noise=None, amp=0.0, dtau=None, want_n_T=False):
        """dL/du0 (and dL/dn0, dL/dT0) of the initial condition given lam_1."""
        g = self.grid_shape
        n0 = self._dev64(n0, g)
        T0 = self._dev64(T0, g)
        u0 = self._dev64(u0, (self.d,) + g)
        if noise is not None:
            noise = self._dev64(noise, (self.Q,) + g)
        du0 = torch.empty((self.d,) + g, dtype=torch.float64, device="cuda")
        dn0 = torch.empty(g, dtype=torch.float64, device="cuda") if want_n_T else None
        dT0 = torch.empty(g, dtype=torch.float64, device="cuda") if want_n_T else None
        _check(lib().rlbm_init_vjp(self.h, _ptr(n0), _ptr(T0), _ptr(u0), _ptr(noise), float(amp), _ptr(lam1),
                                   _ptr(du0), _ptr(dn0), _ptr(dT0), _ptr(dtau), _stream()))
        self._keep_vjp = (n0, T0, u0, noise)
        return (du0, dn0, dT0) if want_n_T else du0

    # launch variants -----------------------------------------------------
    @property
    def variant(self):
        v = c_int32(0)
        _check(lib().rlbm_get_variant(self.h, ctypes.byref(v)))
        return v.value

    @variant.setter
    def variant(self, v):
        _check(lib().rlbm_set_variant(self.h, int(v)))

    STORE_MODES = {"auto": 0, "cached": 1, "nontemporal": 2}

    @property
    def store_mode(self):
        """How the step writes populations: "auto" (non-temporal once both state buffers together exceed
        384 MiB, 1.5 times the last-level cache, and a row of sites is a multiple of 64 bytes), "cached" or "nontemporal" (rlbm_set_store_mode)."""
        m, nt = c_int32(0), c_int32(0)
        _check(lib().rlbm_get_store_mode(self.h, ctypes.byref(m), ctypes.byref(nt)))
        return {v: k for k, v in self.STORE_MODES.items()}[m.value]

    @store_mode.setter
    def store_mode(self, mode):
        _check(lib().rlbm_set_store_mode(self.h, self.STORE_MODES[mode]))

    @property
    def nontemporal_stores(self):
        """Whether the step currently uses non-temporal population stores."""
        m, nt = c_int32(0), c_int32(0)
        _check(lib().rlbm_get_store_mode(self.h, ctypes.byref(m), ctypes.byref(nt)))
        return bool(nt.value)

    def autotune(self, steps=5):
        """Time every launch variant on scratch buffers; keep the fastest. Returns ms per step per variant."""
        n = lib().rlbm_variant_count()
        ms = (ctypes.c_float * n)()
        _check(lib().rlbm_autotune(self.h, int(steps), ms, _stream()))
        return list(ms)


class Batch:
    """Many 2D product-rule lattices advanced by one persistent launch per step (rlbm_batch_*).

    ``specs`` is a list of dicts with keys extent, zeta, tau (and optional bc).
    The state is one flat tensor of ``total_elems`` elements; ``view(f, l)``
    is lattice l's (Q, ny, nx) part of it.  ``member(l)`` is a non-owning
    Lattice over the same handle (its step is the per-lattice launch path)."""

    def __init__(self, specs, order=3, storage="f64"):
        L = lib()
        self.storage = storage
        self.dtype = torch.float64 if storage == "f64" else torch.float32
        n = len(specs)
        cfgs = (Config * n)()
        self.specs = [dict(s) for s in specs]
        for i, sp in enumerate(self.specs):
            c = cfgs[i]
            c.model = _model(2, sp["zeta"], order, "product")
            ext = (int(sp["extent"][0]), int(sp["extent"][1]), 1)
            bc = sp.get("bc", ("periodic", "periodic"))
            for a in range(3):
                c.extent[a] = ext[a]
                c.bc[a] = BC[bc[a]] if a < 2 else 0
            c.storage = STORAGE[storage]
            c.tau = float(sp["tau"])
            c.tau_field = None
            c.n_ref = 1.0
            for a, g in enumerate(sp.get("force", ())):
                c.force[a] = float(g)
        h = c_void_p()
        _check(L.rlbm_batch_create(cfgs, n, ctypes.byref(h)))
        self.h = h
        self.count = n
        te, ts = c_int64(0), c_int64(0)
        eo = (c_int64 * n)()
        so = (c_int64 * n)()
        _check(L.rlbm_batch_layout(h, ctypes.byref(te), ctypes.byref(ts), eo, so))
        self.total_elems, self.total_sites = te.value, ts.value
        self.elem_off, self.site_off = list(eo), list(so)
        self.members = []
        for i, sp in enumerate(self.specs):
            mh = c_void_p()
            _check(L.rlbm_batch_lattice(h, i, ctypes.byref(mh)))
            self.members.append(Lattice(d=2, zeta=sp["zeta"], order=order, extent=sp["extent"],
                                        bc=sp.get("bc"), storage=storage, tau=sp["tau"], force=sp.get("force"),
                                        _handle=mh))
        self.Q = self.members[0].Q

    def __del__(self):
        h = getattr(self, "h", None)
        for m in getattr(self, "members", []):
            m.h = None
        if h is not None and h.value is not None and _lib is not None:
            _lib.rlbm_batch_destroy(h)
        self.h = None

    def new_state(self):
        return torch.empty((self.total_elems,), dtype=self.dtype, device="cuda")

    def view(self, f, l):
        nx, ny = self.members[l].extent
        o = self.elem_off[l]
        return f[o:o + self.Q * nx * ny].view(self.Q, ny, nx)

    def init(self, n0s, T0s, u0s, out=None):
        """Initial post-collision state from per-lattice fields (lists of [ny, nx] / [2, ny, nx] arrays)."""
        cat = lambda xs: torch.cat([torch.as_tensor(x, dtype=torch.float64).reshape(-1) for x in xs]).to("cuda")
        n0, T0, u0 = cat(n0s), cat(T0s), cat(u0s)
        assert n0.numel() == self.total_sites and u0.numel() == 2 * self.total_sites
        out = self.new_state() if out is None else out
        _check(lib().rlbm_batch_init(self.h, _ptr(n0), _ptr(T0), _ptr(u0), _ptr(out), _stream()))
        self._keep = (n0, T0, u0)
        return out

    def step(self, f_a, f_b, nsteps, graph=True):
        assert f_a.dtype == self.dtype and f_b.dtype == self.dtype
        assert f_a.numel() == self.total_elems and f_b.numel() == self.total_elems
        _check(lib().rlbm_batch_step(self.h, _ptr(f_a), _ptr(f_b), int(nsteps), int(bool(graph)), _stream()))
        return f_b if nsteps % 2 == 1 else f_a

    def moments(self, f):
        """Per-lattice fields of the streamed state: list of dicts (views of concatenated arrays)."""
        S = self.total_sites
        dev = "cuda"
        flat = {k: torch.empty(S, dtype=torch.float64, device=dev) for k in ("n", "eps", "T")}
        flat["U"] = torch.empty(3 * S, dtype=torch.float64, device=dev)
        fs = Fields(n=flat["n"].data_ptr(), eps=flat["eps"].data_ptr(), T=flat["T"].data_ptr(),
                    U=flat["U"].data_ptr())
        _check(lib().rlbm_batch_moments(self.h, _ptr(f), ctypes.byref(fs), _stream()))
        out = []
        for l, m in enumerate(self.members):
            nx, ny = m.extent
            so, ns = self.site_off[l], nx * ny
            d = {k: flat[k][so:so + ns].view(ny, nx) for k in ("n", "eps", "T")}
            d["U"] = flat["U"][3 * so:3 * so + 3 * ns].view(3, ny, nx)
            out.append(d)
        return out

    def sync(self):
        _check(lib().rlbm_batch_sync(self.h, _stream()))

    @property
    def variant(self):
        v = c_int32(0)
        _check(lib().rlbm_batch_get_variant(self.h, ctypes.byref(v)))
        return v.value

    @variant.setter
    def variant(self, v):
        _check(lib().rlbm_batch_set_variant(self.h, int(v)))

    @property
    def store_mode(self):
        """"auto", "cached" or "nontemporal" population stores (rlbm_batch_set_store_mode)."""
        m, nt = c_int32(0), c_int32(0)
        _check(lib().rlbm_batch_get_store_mode(self.h, ctypes.byref(m), ctypes.byref(nt)))
        return {v: k for k, v in Lattice.STORE_MODES.items()}[m.value]

    @store_mode.setter
    def store_mode(self, mode):
        _check(lib().rlbm_batch_set_store_mode(self.h, Lattice.STORE_MODES[mode]))

    @property
    def nontemporal_stores(self):
        m, nt = c_int32(0), c_int32(0)
        _check(lib().rlbm_batch_get_store_mode(self.h, ctypes.byref(m), ctypes.byref(nt)))
        return bool(nt.value)

    def autotune(self, f_a, f_b, steps=4):
        """Time every batch variant on (f_a, f_b) (state ends in f_a); keep the fastest."""
        n = lib().rlbm_batch_variant_count()
        ms = (ctypes.c_float * n)()
        _check(lib().rlbm_batch_autotune(self.h, _ptr(f_a), _ptr(f_b), int(steps), ms, _stream()))
        return list(ms)
