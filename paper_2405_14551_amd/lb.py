"""ctypes binding of the C ABI in ``include/lb.h`` (argument marshalling only).

Every step of the path runs in the HIP library ``liblbmi.so``; this module
converts Python arguments, allocates caller-owned output tensors with
PyTorch (device memory) and passes the current PyTorch stream.  If the
library is missing it raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
# LB_LIBRARY: a library built with other compile-time settings
LIB_PATH = os.environ.get("LB_LIBRARY", os.path.join(PKG, "liblbmi.so"))

LB_OK, LB_EINVAL, LB_ENOMEM, LB_EHIP, LB_ENUMERIC, LB_ENODEV, LB_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
LATTICE = {"D2Q9": 0, "D3Q19": 1, "D3Q27": 2}
STORAGE = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3, "f32t": 4, "f16t": 5, "bf16t": 6, "f16ct": 7, "f32s": 8}
TOTAL_LAYOUTS = ("f32t", "f16t", "bf16t", "f16ct")
NC_MODE = {"off": 0, "explicit": 1, "mlp": 2}
STREAMING = {"two_copies": 0, "in_place": 1}
SCHEME = {"populations": 0, "moments": 1}
ROUNDING = {"nearest": 0, "stochastic": 1}
PHASE_PASS = {"auto": 0, "scatter": 1, "pass": 2}
N_MOMENTS = 15
MLP_PARAMS = 6339
MLP_ROW = 32
FIELD_BITS = {"rho_a": 0, "rho_b": 1, "phi": 2, "u": 3, "f_nc": 4, "flags": 5, "labels": 6}
Q_OF = {"D2Q9": 9, "D3Q19": 19, "D3Q27": 27}



class LBError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


class LbTuning(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("z_per_block", ctypes.c_int), ("use_graph", ctypes.c_int),
                ("reserved", ctypes.c_int), ("ms_per_step", ctypes.c_double)]


ENSEMBLE_MODE = {"batched": 0, "per_channel": 1}
ENSEMBLE_MODE_NAME = {v: k for k, v in ENSEMBLE_MODE.items()}


class LbParams(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int), ("storage", ctypes.c_int), ("nc_mode", ctypes.c_int),
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("wall", ctypes.c_int * 3),
        ("tau", ctypes.c_double), ("A", ctypes.c_double), ("beta", ctypes.c_double),
        ("rho0", ctypes.c_double),
        ("body_force", ctypes.c_double * 3), ("u0", ctypes.c_double * 3),
        ("nc_A", ctypes.c_double), ("nc_hmin", ctypes.c_double), ("nc_hmax", ctypes.c_double),
        ("phi_interface", ctypes.c_double),
        ("diag_every", ctypes.c_int),
        ("streaming", ctypes.c_int),
        ("tau_b", ctypes.c_double),
        ("scheme", ctypes.c_int),
        ("rounding", ctypes.c_int),
        ("phase_pass", ctypes.c_int),
    ]


_lib = None

EXPORTED = [
    "lb_params_default", "lb_create", "lb_init_droplets", "lb_step", "lb_fields",
    "lb_diagnostics", "lb_state_bytes", "lb_get_state", "lb_set_state", "lb_step_count",
    "lb_sync", "lb_destroy", "lb_lattice_table", "lb_error_string", "lb_last_error",
    "lb_profile_begin", "lb_profile_end", "lb_channel_count", "lb_get_tuning", "lb_set_tuning",
    "lb_autotune", "lb_nc_collect", "lb_nc_collect_noalloc", "lb_mlp_set_weights", "lb_mlp_get_weights",
    "lb_mlp_set_ranges", "lb_mlp_get_ranges", "lb_mlp_train", "lb_mlp_gradient", "lb_mlp_infer",
]


def lib():
    """Load liblbmi.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2405_14551_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    P = ctypes.POINTER
    L.lb_params_default.argtypes = [P(LbParams)]
    L.lb_params_default.restype = None
    L.lb_create.argtypes = [P(LbParams), i, vp, P(vp)]
    L.lb_init_droplets.argtypes = [vp, i, i, P(d), P(d), d, d]
    L.lb_step.argtypes = [vp, i]
    L.lb_fields.argtypes = [vp, i, ctypes.c_uint, P(vp), i]
    L.lb_diagnostics.argtypes = [vp, i, P(d)]
    L.lb_state_bytes.argtypes = [vp, P(sz)]
    L.lb_get_state.argtypes = [vp, vp, sz, i]
    L.lb_set_state.argtypes = [vp, vp, sz, i]
    L.lb_step_count.argtypes = [vp, P(ctypes.c_longlong)]
    L.lb_sync.argtypes = [vp]
    L.lb_destroy.argtypes = [vp]
    L.lb_lattice_table.argtypes = [i, P(i), P(i), P(d), P(i), P(d)]
    L.lb_profile_begin.argtypes = [vp]
    L.lb_profile_end.argtypes = [vp, P(d), P(d), P(d), P(i), P(i), P(i)]
    L.lb_channel_count.argtypes = [vp, P(i)]
    L.lb_get_tuning.argtypes = [vp, P(LbTuning)]
    L.lb_set_tuning.argtypes = [vp, P(LbTuning)]
    L.lb_autotune.argtypes = [vp, i, P(LbTuning), P(d), i, P(i)]
    ll = ctypes.c_longlong
    fp = P(ctypes.c_float)
    L.lb_nc_collect.argtypes = [vp, i, vp, vp, ll, P(ll), P(ll)]
    L.lb_nc_collect_noalloc.argtypes = [vp, i, vp, vp, ll, P(ll), P(ll)]
    L.lb_mlp_set_weights.argtypes = [vp, fp, ll]
    L.lb_mlp_get_weights.argtypes = [vp, fp, ll]
    L.lb_mlp_set_ranges.argtypes = [vp, fp, fp, ctypes.c_float]
    L.lb_mlp_get_ranges.argtypes = [vp, fp, fp, fp]
    L.lb_mlp_train.argtypes = [vp, vp, vp, ll, vp, i, i, d, vp]
    L.lb_mlp_gradient.argtypes = [vp, vp, vp, ll, vp, vp]
    L.lb_mlp_infer.argtypes = [vp, vp, vp, ll]
    L.lb_error_string.argtypes = [i]
    L.lb_error_string.restype = ctypes.c_char_p
    L.lb_last_error.argtypes = []
    L.lb_last_error.restype = ctypes.c_char_p
    for name in ["lb_create", "lb_init_droplets", "lb_step", "lb_fields", "lb_diagnostics",
                 "lb_state_bytes", "lb_get_state", "lb_set_state", "lb_step_count", "lb_sync",
                 "lb_destroy", "lb_lattice_table", "lb_profile_begin", "lb_profile_end",
                 "lb_channel_count", "lb_get_tuning", "lb_set_tuning", "lb_autotune", "lb_nc_collect",
                 "lb_nc_collect_noalloc", "lb_mlp_set_weights", "lb_mlp_get_weights", "lb_mlp_set_ranges", "lb_mlp_get_ranges",
                 "lb_mlp_train", "lb_mlp_gradient", "lb_mlp_infer"]:
        getattr(L, name).restype = i
    _lib = L
    return L


def check(code):
    if code != LB_OK:
        L = lib()
        raise LBError(code, f"{L.lb_error_string(code).decode()}: {L.lb_last_error().decode()}")
    return code


def lattice_table(name):
    """(c int[q,3], w float64[q], opp int[q], B float64[q]) as the library defines them."""
    L = lib()
    q = Q_OF[name]
    qq = ctypes.c_int()
    c = (ctypes.c_int * (3 * q))()
    w = (ctypes.c_double * q)()
    o = (ctypes.c_int * q)()
    B = (ctypes.c_double * q)()
    check(L.lb_lattice_table(LATTICE[name], ctypes.byref(qq), c, w, o, B))
    return (np.array(c[:], dtype=np.int64).reshape(q, 3), np.array(w[:]), np.array(o[:], dtype=np.int64),
            np.array(B[:]))


def make_params(lattice="D3Q27", storage="f32", nc="off", shape=(64, 64, 64), walls=(0, 0, 0),
                tau=1.0, A=0.01, beta=0.7, rho0=1.0, body_force=(0.0, 0.0, 0.0), u0=(0.0, 0.0, 0.0),
                nc_A=0.02, nc_hmin=2.0, nc_hmax=3.0, phi_interface=0.9, diag_every=0,
                streaming="two_copies", tau_b=0.0, scheme="populations", rounding="nearest", phase="auto"):
    p = LbParams()
    lib().lb_params_default(ctypes.byref(p))
    p.lattice = LATTICE[lattice]
    p.storage = STORAGE[storage]
    p.nc_mode = NC_MODE[nc] if isinstance(nc, str) else (1 if nc else 0)
    p.nx, p.ny, p.nz = (int(v) for v in shape)
    for a in range(3):
        p.wall[a] = int(bool(walls[a]))
        p.body_force[a] = float(body_force[a])
        p.u0[a] = float(u0[a])
    p.tau, p.A, p.beta, p.rho0 = float(tau), float(A), float(beta), float(rho0)
    p.nc_A, p.nc_hmin, p.nc_hmax = float(nc_A), float(nc_hmin), float(nc_hmax)
    p.phi_interface = float(phi_interface)
    p.diag_every = int(diag_every)
    p.streaming = STREAMING[streaming]
    p.tau_b = float(tau_b)
    p.scheme = SCHEME[scheme]
    p.rounding = ROUNDING[rounding]
    p.phase_pass = PHASE_PASS[phase]
    return p


class Simulation:
    """One lattice on the current GPU.  Fields come back as torch tensors of
    shape (nz, ny, nx) or (3, nz, ny, nx)."""

    def __init__(self, lattice="D3Q27", storage="f32", nc="off", shape=(64, 64, 64), stream=None,
                 **kw):
        import torch
        self.torch = torch
        self.lattice = lattice
        self.storage = storage
        self.shape = tuple(int(v) for v in shape)
        self.q = Q_OF[lattice]
        self.params = make_params(lattice, storage, nc, shape, **kw)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.device = torch.device("cuda", torch.cuda.current_device())
        h = ctypes.c_void_p()
        check(lib().lb_create(ctypes.byref(self.params), 1, ctypes.c_void_p(stream.cuda_stream),
                              ctypes.byref(h)))
        self.h = h
        self.real = torch.float64 if storage == "f64" else torch.float32
        self.state_dtype = {"f64": torch.float64, "f32": torch.float32, "f16": torch.float16,
                            "bf16": torch.bfloat16, "f32t": torch.float32, "f16t": torch.float16,
                            "bf16t": torch.bfloat16, "f16ct": torch.int16, "f32s": torch.float32}[storage]
        self.total = storage in TOTAL_LAYOUTS
        self.moments = kw.get("scheme", "populations") == "moments"

    # -------------------------------------------------------------- lifetime
    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            check(lib().lb_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ---------------------------------------------------------------- calls
    def init_droplets(self, centres, radii, width=2.0, phi_in=1.0):
        c = np.ascontiguousarray(np.asarray(centres, dtype=np.float64).reshape(-1, 3))
        r = np.ascontiguousarray(np.asarray(radii, dtype=np.float64).reshape(-1))
        if c.shape[0] != r.shape[0]:
            raise ValueError("centres and radii differ in length")
        dp = ctypes.POINTER(ctypes.c_double)
        check(lib().lb_init_droplets(self.h, 0, int(r.shape[0]), c.ctypes.data_as(dp),
                                     r.ctypes.data_as(dp), float(width), float(phi_in)))
        return self

    def step(self, n=1):
        check(lib().lb_step(self.h, int(n)))
        return self

    def sync(self):
        check(lib().lb_sync(self.h))

    def set_z_per_block(self, zb):
        """Planes per collision march (lb_set_tuning on a single lattice)."""
        t = LbTuning()
        check(lib().lb_get_tuning(self.h, ctypes.byref(t)))
        t.z_per_block = int(zb)
        check(lib().lb_set_tuning(self.h, ctypes.byref(t)))
        return self

    def tuning(self):
        """dict(z_per_block, use_graph) of this lattice (lb_get_tuning)."""
        t = LbTuning()
        check(lib().lb_get_tuning(self.h, ctypes.byref(t)))
        return {"z_per_block": t.z_per_block, "use_graph": t.use_graph}

    def autotune(self, steps=4):
        """Time z-planes per march {1, 2, 4, 8, 16, 32} (up to nz) with and without
        graph replays (the timed steps advance the simulation), keep the
        fastest and return (best, table) (lb_autotune)."""
        best = LbTuning()
        cap = 64
        res = (ctypes.c_double * (4 * cap))()
        n = ctypes.c_int()
        check(lib().lb_autotune(self.h, int(steps), ctypes.byref(best), res, cap, ctypes.byref(n)))
        table = [{"z_per_block": int(res[4 * k + 1]), "use_graph": int(res[4 * k + 2]), "ms_per_step": res[4 * k + 3]}
                 for k in range(min(n.value, cap))]
        return {"z_per_block": best.z_per_block, "use_graph": best.use_graph, "ms_per_step": best.ms_per_step}, table

    def set_graph(self, on=True):
        """Replay pairs of non-field steps from a captured hipGraph
        (lb_tuning.use_graph on a single lattice)."""
        t = LbTuning()
        check(lib().lb_get_tuning(self.h, ctypes.byref(t)))
        t.use_graph = int(bool(on))
        check(lib().lb_set_tuning(self.h, ctypes.byref(t)))
        return self

    def profile_begin(self):
        check(lib().lb_profile_begin(self.h))

    def profile_end(self):
        """Returns dict(ms_phase, ms_collide, ms_combine, n_phase, n_collide, n_combine)
        summed over launches (combine: the read-once step's second launch)."""
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        na, nb, nc = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        check(lib().lb_profile_end(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(na),
                                   ctypes.byref(nb), ctypes.byref(nc)))
        return dict(ms_phase=a.value, ms_collide=b.value, ms_combine=c.value, n_phase=na.value,
                    n_collide=nb.value, n_combine=nc.value)

    @property
    def t(self):
        v = ctypes.c_longlong()
        check(lib().lb_step_count(self.h, ctypes.byref(v)))
        return v.value

    def fields(self, names=("rho_a", "rho_b", "phi", "u", "f_nc", "flags")):
        torch = self.torch
        nx, ny, nz = self.shape
        out = {}
        ptrs = (ctypes.c_void_p * 7)()
        mask = 0
        for nm in names:
            b = FIELD_BITS[nm]
            if nm in ("u", "f_nc"):
                t = torch.empty((3, nz, ny, nx), dtype=self.real, device=self.device)
            elif nm == "flags":
                t = torch.empty((nz, ny, nx), dtype=torch.uint8, device=self.device)
            elif nm == "labels":
                t = torch.empty((nz, ny, nx), dtype=torch.int32, device=self.device)
            else:
                t = torch.empty((nz, ny, nx), dtype=self.real, device=self.device)
            out[nm] = t
            ptrs[b] = t.data_ptr()
            mask |= 1 << b
        check(lib().lb_fields(self.h, 0, mask, ptrs, 1))
        self.stream.synchronize()
        return out

    def diagnostics(self):
        d = (ctypes.c_double * 8)()
        check(lib().lb_diagnostics(self.h, 0, d))
        return np.array(d[:])

    def state_bytes(self):
        v = ctypes.c_size_t()
        check(lib().lb_state_bytes(self.h, ctypes.byref(v)))
        return v.value

    def get_state(self, host=False):
        """Post-collision state on the device.  Per-colour layouts: a tensor
        (2, q, nz, ny, nx) of the storage type.  Total layouts: a uint8 tensor
        of the raw bytes (use ``split_total_state``).  Moment scheme: a tensor
        (15, nz, ny, nx) of the moments (channel 0 holds rho - rho0).  host=True: the raw bytes
        as a numpy uint8 array, copied by the library to host memory."""
        nx, ny, nz = self.shape
        if host:
            a = np.empty((self.state_bytes(),), dtype=np.uint8)
            check(lib().lb_get_state(self.h, ctypes.c_void_p(a.ctypes.data), a.nbytes, 0))
            return a
        if self.total:
            t = self.torch.empty((self.state_bytes(),), dtype=self.torch.uint8, device=self.device)
        elif self.moments:
            t = self.torch.empty((N_MOMENTS, nz, ny, nx), dtype=self.state_dtype, device=self.device)
        else:
            t = self.torch.empty((2, self.q, nz, ny, nx), dtype=self.state_dtype, device=self.device)
        check(lib().lb_get_state(self.h, ctypes.c_void_p(t.data_ptr()), self.state_bytes(), 1))
        self.stream.synchronize()
        return t

    def split_total_state(self, raw):
        """(T (q, nz, ny, nx) in the storage type, scalars (4, nz, ny, nx) float32)
        views of a total-layout state."""
        nx, ny, nz = self.shape
        n = self.q * nx * ny * nz * self.torch.tensor([], dtype=self.state_dtype).element_size()
        T = raw[:n].view(self.state_dtype).view(self.q, nz, ny, nx)
        sc = raw[n:].view(self.torch.float32).view(4, nz, ny, nx)
        return T, sc

    def set_state(self, t):
        if self.total:
            t = t.to(device=self.device).contiguous().view(self.torch.uint8).reshape(-1)
        else:
            t = t.to(device=self.device, dtype=self.state_dtype).contiguous()
        if t.numel() * t.element_size() != self.state_bytes():
            raise ValueError("state has the wrong size")
        self.stream.synchronize()
        check(lib().lb_set_state(self.h, ctypes.c_void_p(t.data_ptr()), self.state_bytes(), 1))
        self.stream.synchronize()
        return self

    # ---------------------------------------------------- learned closure
    def _dev_f32(self, t, cols):
        t = self.torch.as_tensor(t).to(device=self.device, dtype=self.torch.float32).contiguous()
        if t.dim() != 2 or t.shape[1] != cols:
            raise ValueError(f"expected an (m, {cols}) array")
        return t

    def nc_collect(self):
        """Training rows of the last (explicit-force) step: (rows (m, 32),
        targets (m, 3), m_active, m_free) as float32 device tensors, active
        rows first."""
        L = lib()
        na, nf = ctypes.c_longlong(), ctypes.c_longlong()
        check(L.lb_nc_collect(self.h, 0, None, None, 0, ctypes.byref(na), ctypes.byref(nf)))
        m = na.value + nf.value
        rows = self.torch.empty((max(m, 1), MLP_ROW), dtype=self.torch.float32, device=self.device)
        tg = self.torch.empty((max(m, 1), 3), dtype=self.torch.float32, device=self.device)
        check(L.lb_nc_collect(self.h, 0, ctypes.c_void_p(rows.data_ptr()), ctypes.c_void_p(tg.data_ptr()), m,
                              ctypes.byref(na), ctypes.byref(nf)))
        return rows[:m], tg[:m], na.value, nf.value

    def nc_collect_into(self, rows, targets):
        """Allocation-free collection into caller-owned float32 device tensors
        rows (cap, 32) and targets (cap, 3): the library allocates no device
        memory for it.  Rows beyond cap are not written.  Returns (m_active,
        m_free)."""
        if rows.dtype != self.torch.float32 or targets.dtype != self.torch.float32:
            raise ValueError("rows and targets must be float32")
        if not (rows.is_contiguous() and targets.is_contiguous()):
            raise ValueError("rows and targets must be contiguous")
        if rows.dim() != 2 or rows.shape[1] != MLP_ROW or targets.dim() != 2 or targets.shape[1] != 3 \
                or targets.shape[0] != rows.shape[0]:
            raise ValueError(f"expected rows (cap, {MLP_ROW}) and targets (cap, 3)")
        na, nf = ctypes.c_longlong(), ctypes.c_longlong()
        check(lib().lb_nc_collect_noalloc(self.h, 0, ctypes.c_void_p(rows.data_ptr()),
                                          ctypes.c_void_p(targets.data_ptr()), rows.shape[0],
                                          ctypes.byref(na), ctypes.byref(nf)))
        return na.value, nf.value

    def mlp_set_weights(self, theta):
        th = np.ascontiguousarray(np.asarray(theta, dtype=np.float32).reshape(-1))
        check(lib().lb_mlp_set_weights(self.h, th.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), th.size))
        return self

    def mlp_get_weights(self):
        th = np.empty(MLP_PARAMS, dtype=np.float32)
        check(lib().lb_mlp_get_weights(self.h, th.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), th.size))
        return th

    def mlp_set_ranges(self, lo, hi, gmin):
        fp = ctypes.POINTER(ctypes.c_float)
        lo = np.ascontiguousarray(np.asarray(lo, dtype=np.float32).reshape(30))
        hi = np.ascontiguousarray(np.asarray(hi, dtype=np.float32).reshape(30))
        check(lib().lb_mlp_set_ranges(self.h, lo.ctypes.data_as(fp), hi.ctypes.data_as(fp), float(gmin)))
        return self

    def mlp_get_ranges(self):
        fp = ctypes.POINTER(ctypes.c_float)
        lo, hi, g = np.empty(30, np.float32), np.empty(30, np.float32), np.empty(1, np.float32)
        check(lib().lb_mlp_get_ranges(self.h, lo.ctypes.data_as(fp), hi.ctypes.data_as(fp), g.ctypes.data_as(fp)))
        return lo, hi, g[0]

    def mlp_train(self, rows, targets, order, lr=1e-3):
        """Adam over the mini-batches order[t] (int32 (n_steps, batch) row
        indices); returns the per-step batch losses (float32 device tensor)."""
        torch = self.torch
        rows = self._dev_f32(rows, MLP_ROW)
        targets = self._dev_f32(targets, 3)
        order = torch.as_tensor(order).to(device=self.device, dtype=torch.int32).contiguous()
        n_steps, batch = order.shape
        log = torch.empty(max(n_steps, 1), dtype=torch.float32, device=self.device)
        self.stream.synchronize()
        check(lib().lb_mlp_train(self.h, ctypes.c_void_p(rows.data_ptr()), ctypes.c_void_p(targets.data_ptr()),
                                 rows.shape[0], ctypes.c_void_p(order.data_ptr()), n_steps, batch, float(lr),
                                 ctypes.c_void_p(log.data_ptr())))
        return log[:n_steps]

    def mlp_gradient(self, rows, targets):
        """(loss, gradient) of the mean squared error over all rows."""
        torch = self.torch
        rows = self._dev_f32(rows, MLP_ROW)
        targets = self._dev_f32(targets, 3)
        g = torch.empty(MLP_PARAMS, dtype=torch.float32, device=self.device)
        l = torch.empty(1, dtype=torch.float32, device=self.device)
        self.stream.synchronize()
        check(lib().lb_mlp_gradient(self.h, ctypes.c_void_p(rows.data_ptr()), ctypes.c_void_p(targets.data_ptr()),
                                    rows.shape[0], ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(l.data_ptr())))
        return float(l.item()), g

    def mlp_infer(self, rows):
        rows = self._dev_f32(rows, MLP_ROW)
        out = self.torch.empty((rows.shape[0], 3), dtype=self.torch.float32, device=self.device)
        self.stream.synchronize()
        check(lib().lb_mlp_infer(self.h, ctypes.c_void_p(rows.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                 rows.shape[0]))
        self.stream.synchronize()
        return out


def _tuning_dict(t):
    return {"mode": ENSEMBLE_MODE_NAME[t.mode], "z_per_block": t.z_per_block, "use_graph": t.use_graph,
            "ms_per_step": t.ms_per_step}


class Ensemble:
    """Independent lattices ("channels") advanced together by batched
    launches (one phase and one collision launch over all channels' tiles per
    step, or the single-lattice launches channel after channel; see
    ``set_tuning``).  ``channels`` is a list of dicts of per-channel
    parameters (shape, walls, tau, A, beta, body_force, ...); lattice, storage
    and nc are shared."""

    def __init__(self, channels, lattice="D3Q19", storage="f32", nc="explicit", stream=None):
        import torch
        self.torch = torch
        self.lattice = lattice
        self.storage = storage
        self.q = Q_OF[lattice]
        self.shapes = [tuple(int(v) for v in c["shape"]) for c in channels]
        arr = (LbParams * len(channels))()
        for k, c in enumerate(channels):
            kw = {key: v for key, v in c.items() if key != "shape"}
            arr[k] = make_params(lattice, storage, nc, c["shape"], **kw)
        self._params = arr
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.device = torch.device("cuda", torch.cuda.current_device())
        h = ctypes.c_void_p()
        check(lib().lb_create(arr, len(channels), ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
        self.h = h
        self.real = torch.float64 if storage == "f64" else torch.float32
        self.total = storage in TOTAL_LAYOUTS

    @property
    def n_channels(self):
        return len(self.shapes)

    @property
    def sites(self):
        return sum(a * b * c for a, b, c in self.shapes)

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            check(lib().lb_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_droplets(self, channel, centres, radii, width=2.0, phi_in=1.0):
        c = np.ascontiguousarray(np.asarray(centres, dtype=np.float64).reshape(-1, 3))
        r = np.ascontiguousarray(np.asarray(radii, dtype=np.float64).reshape(-1))
        dp = ctypes.POINTER(ctypes.c_double)
        check(lib().lb_init_droplets(self.h, int(channel), int(r.shape[0]), c.ctypes.data_as(dp),
                                     r.ctypes.data_as(dp), float(width), float(phi_in)))
        return self

    def step(self, n=1):
        check(lib().lb_step(self.h, int(n)))
        return self

    def sync(self):
        check(lib().lb_sync(self.h))

    def fields(self, channel, names=("rho_a", "rho_b", "phi", "u", "f_nc", "flags")):
        torch = self.torch
        nx, ny, nz = self.shapes[channel]
        out = {}
        ptrs = (ctypes.c_void_p * 7)()
        mask = 0
        for nm in names:
            b = FIELD_BITS[nm]
            if nm in ("u", "f_nc"):
                t = torch.empty((3, nz, ny, nx), dtype=self.real, device=self.device)
            elif nm == "flags":
                t = torch.empty((nz, ny, nx), dtype=torch.uint8, device=self.device)
            elif nm == "labels":
                t = torch.empty((nz, ny, nx), dtype=torch.int32, device=self.device)
            else:
                t = torch.empty((nz, ny, nx), dtype=self.real, device=self.device)
            out[nm] = t
            ptrs[b] = t.data_ptr()
            mask |= 1 << b
        check(lib().lb_fields(self.h, int(channel), mask, ptrs, 1))
        self.stream.synchronize()
        return out

    def diagnostics(self, channel):
        d = (ctypes.c_double * 8)()
        check(lib().lb_diagnostics(self.h, int(channel), d))
        return np.array(d[:])

    def state_bytes(self):
        v = ctypes.c_size_t()
        check(lib().lb_state_bytes(self.h, ctypes.byref(v)))
        return v.value

    def get_state(self):
        """Raw state bytes (uint8 device tensor): the channels' states in order."""
        t = self.torch.empty((self.state_bytes(),), dtype=self.torch.uint8, device=self.device)
        check(lib().lb_get_state(self.h, ctypes.c_void_p(t.data_ptr()), self.state_bytes(), 1))
        self.stream.synchronize()
        return t

    def set_state(self, raw):
        raw = raw.to(device=self.device).contiguous().view(self.torch.uint8).reshape(-1)
        if raw.numel() != self.state_bytes():
            raise ValueError("state has the wrong size")
        self.stream.synchronize()
        check(lib().lb_set_state(self.h, ctypes.c_void_p(raw.data_ptr()), self.state_bytes(), 1))
        self.stream.synchronize()
        return self

    def channel_state(self, raw, channel):
        """(2, q, nz, ny, nx) view of one channel's per-colour state inside ``raw``."""
        es = self.torch.tensor([], dtype=self.real).element_size()
        off = 0
        for k, (nx, ny, nz) in enumerate(self.shapes):
            n = 2 * self.q * nx * ny * nz * es
            if k == channel:
                return raw[off:off + n].view(self.real).view(2, self.q, nz, ny, nx)
            off += n
        raise IndexError(channel)

    def tuning(self):
        t = LbTuning()
        check(lib().lb_get_tuning(self.h, ctypes.byref(t)))
        return _tuning_dict(t)

    def set_tuning(self, mode="batched", z_per_block=4, use_graph=1):
        t = LbTuning(ENSEMBLE_MODE[mode], int(z_per_block), int(use_graph), 0, 0.0)
        check(lib().lb_set_tuning(self.h, ctypes.byref(t)))
        return self

    def autotune(self, steps=4, cache=None):
        """Time every candidate configuration (the timed steps advance the
        simulation), keep the fastest and return (best, table).  With ``cache``
        (a JSON path) the choice is stored there and reused when present."""
        import json
        import os
        key = f"{self.lattice}/{self.storage}/{self.n_channels}ch/{self.sites}sites"
        if cache and os.path.exists(cache):
            stored = json.load(open(cache))
            if key in stored:
                b = stored[key]["best"]
                self.set_tuning(b["mode"], b["z_per_block"], b["use_graph"])
                return b, stored[key]["table"]
        best = LbTuning()
        cap = 64
        res = (ctypes.c_double * (4 * cap))()
        n = ctypes.c_int()
        check(lib().lb_autotune(self.h, int(steps), ctypes.byref(best), res, cap, ctypes.byref(n)))
        table = [{"mode": ENSEMBLE_MODE_NAME[int(res[4 * k])], "z_per_block": int(res[4 * k + 1]),
                  "use_graph": int(res[4 * k + 2]), "ms_per_step": res[4 * k + 3]}
                 for k in range(min(n.value, cap))]
        b = _tuning_dict(best)
        if cache:
            stored = json.load(open(cache)) if os.path.exists(cache) else {}
            stored[key] = {"best": b, "table": table}
            with open(cache, "w") as fh:
                json.dump(stored, fh, indent=1)
        return b, table

    def profile_begin(self):
        check(lib().lb_profile_begin(self.h))

    def profile_end(self):
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        na, nb, nc = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        check(lib().lb_profile_end(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(na),
                                   ctypes.byref(nb), ctypes.byref(nc)))
        return dict(ms_phase=a.value, ms_collide=b.value, ms_combine=c.value, n_phase=na.value,
                    n_collide=nb.value, n_combine=nc.value)
