"""Python binding of libnks (nested Krylov-Ritz sgn(A) b on MI355X).

Argument marshalling only: every step of the method runs in the HIP kernels
of ``libnks.so``.  PyTorch supplies device memory and the current stream.

    import torch, paper_0912_4457_amd as nks
    ctx = nks.Context()
    lat = nks.Lattice(ctx, dims, links)          # links: complex128 CUDA tensor
    lat.set_params(m0=1.6, mu=0.0)
    x, st = nks.sign_apply(lat, b, k=200, ell=50)

Vector layout: complex128, ``12*site + 3*spin + colour`` with
``site = x + Lx*(y + Ly*(z + Lz*t))``; links ``((site*4 + nu)*3 + row)*3 + col``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = [
    "FP64", "MIXED", "POLICY_FIXED", "POLICY_DOUBLING", "POLICY_LEARNED",
    "NKSError", "lib", "Context", "Lattice", "apply_op", "sign_apply", "sign_apply_batch",
    "outer_basis", "nested_step", "workspace_size", "LIB_PATH", "policy_load", "policy_label", "load_policy",
    "overlap_apply",
    "mlp_forward", "mlp_backward", "mlp_adam_step",
]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libnks.so")

FP64, MIXED = 0, 1
POLICY_FIXED, POLICY_DOUBLING, POLICY_LEARNED = 0, 1, 2
_PREC = {"fp64": FP64, "mixed": MIXED, FP64: FP64, MIXED: MIXED}

STATUS = {0: "ok", 1: "invalid", 2: "nomem", 3: "hip", 4: "unsupported", 5: "breakdown", 6: "noconv"}


class NKSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libnks error {code} ({STATUS.get(code, '?')}): {msg}")
        self.code = code


MAX_LEVELS = 6   # NKS_MAX_LEVELS


class Opts(ctypes.Structure):
    _fields_ = [
        ("size", ctypes.c_size_t), ("k", ctypes.c_int), ("ell", ctypes.c_int), ("tol", ctypes.c_double),
        ("precision", ctypes.c_int), ("p", ctypes.c_double), ("k_policy", ctypes.c_int),
        ("ell_policy", ctypes.c_int), ("max_rhi_iter", ctypes.c_int), ("rhi_tol", ctypes.c_double),
        ("flags", ctypes.c_uint), ("levels", ctypes.c_int),
        ("ell_deep", ctypes.c_int * (MAX_LEVELS - 1)), ("p_deep", ctypes.c_double * (MAX_LEVELS - 1)),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int), ("k_used", ctypes.c_int), ("ell_used", ctypes.c_int),
        ("rhi_iters", ctypes.c_int), ("p_used", ctypes.c_double), ("z_min", ctypes.c_double),
        ("z_max", ctypes.c_double), ("b_norm", ctypes.c_double), ("breakdown_iter", ctypes.c_int),
        ("inner_delta", ctypes.c_double), ("outer_delta", ctypes.c_double),
        ("ms_outer", ctypes.c_float), ("ms_nested", ctypes.c_float), ("ms_lift", ctypes.c_float),
        ("levels_used", ctypes.c_int), ("ell_deep_used", ctypes.c_int * (MAX_LEVELS - 1)),
        ("p_deep_used", ctypes.c_double * (MAX_LEVELS - 1)),
    ]

    def as_dict(self):
        d = {name: getattr(self, name) for name, _ in self._fields_}
        d["ell_deep_used"] = list(self.ell_deep_used)[:max(self.levels_used - 1, 0)]
        d["p_deep_used"] = list(self.p_deep_used)[:max(self.levels_used - 1, 0)]
        d["status_str"] = STATUS.get(self.status, "?")
        return d


class Job(ctypes.Structure):
    _fields_ = [("lat", ctypes.c_void_p), ("b", ctypes.c_void_p), ("x", ctypes.c_void_p),
                ("opts", ctypes.POINTER(Opts))]


# exported symbols and their C signatures (kept in sync with include/nks.h)
_VP, _I, _D, _SZ = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
_PD = ctypes.POINTER(ctypes.c_double)
SIGNATURES = {
    "nks_opts_default": (None, [ctypes.POINTER(Opts)]),
    "nks_create": (_I, [_I, ctypes.POINTER(_VP)]),
    "nks_destroy": (None, [_VP]),
    "nks_last_error": (ctypes.c_char_p, [_VP]),
    "nks_status_str": (ctypes.c_char_p, [_I]),
    "nks_lattice_create": (_I, [_VP, ctypes.POINTER(ctypes.c_int32), _VP, ctypes.POINTER(_VP)]),
    "nks_lattice_set_params": (_I, [_VP, _D, _D]),
    "nks_lattice_destroy": (None, [_VP]),
    "nks_lattice_set_deflation": (_I, [_VP, _I, _VP, _VP, _PD]),
    "nks_lattice_eigensolve": (_I, [_VP, _I, _I, _D, _PD, _PD, ctypes.POINTER(_I)]),
    "nks_lattice_get_deflation": (_I, [_VP, ctypes.POINTER(_I), _VP, _VP]),
    "nks_apply_op": (_I, [_VP, _VP, _VP, _I, _I, _VP]),
    "nks_workspace_size": (_I, [_VP, _I, ctypes.POINTER(Job), ctypes.POINTER(_SZ)]),
    "nks_sign_apply": (_I, [_VP, _VP, _VP, _VP, ctypes.POINTER(Opts), _VP, _SZ, _VP, ctypes.POINTER(Stats)]),
    "nks_sign_apply_batch": (_I, [_VP, _I, ctypes.POINTER(Job), _VP, _SZ, _VP, ctypes.POINTER(Stats)]),
    "nks_sign_apply_noalloc": (_I, [_VP, _VP, _VP, _VP, ctypes.POINTER(Opts), _VP, ctypes.POINTER(Stats)]),
    "nks_outer_basis": (_I, [_VP, _VP, _VP, ctypes.POINTER(Opts), _VP, _SZ, _VP, _PD, _PD, _PD,
                             ctypes.POINTER(Stats)]),
    "nks_nested_step": (_I, [_VP, _I, _PD, _PD, _PD, _I, ctypes.POINTER(Opts), _PD, ctypes.POINTER(Stats)]),
    "nks_mlp_forward": (_I, [_VP, _VP, _VP, _I, _VP, _VP]),
    "nks_mlp_backward": (_I, [_VP, _VP, _VP, _VP, _I, _VP, _VP, _VP]),
    "nks_mlp_adam_step": (_I, [_VP, _VP, _VP, _VP, _VP, _I, ctypes.c_float, _VP]),
    "nks_policy_load": (_I, [_VP, _VP, _I]),
    "nks_policy_label": (_I, [_VP, _I, ctypes.POINTER(Job), _PD]),
    "nks_tune_set": (_I, [_VP, ctypes.c_char_p, _I]),
    "nks_tune_get": (_I, [_VP, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int)]),
    "nks_profile_enable": (_I, [_VP, _I]),
    "nks_profile_read": (_I, [_VP, _I, ctypes.POINTER(ctypes.c_int), _PD, _PD]),
}

KERNEL_CLASSES = {"stencil": 0, "recurrence": 1, "nested": 2, "lift": 3}

_LIB = None


def lib():
    """Load libnks.so (built in-tree); raises if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_0912_4457_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libnks needs a ROCm GPU (torch.cuda.is_available() is False)")
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


FLAG_OVERLAP = 1
FLAG_DEFLATE = 2
FLAG_DOUBLE_PASS = 4


def make_opts(k=200, ell=50, tol=1e-8, precision="fp64", p=None, max_rhi_iter=50, rhi_tol=1e-14,
              k_policy=POLICY_FIXED, ell_policy=POLICY_FIXED, overlap=False, deflate=False,
              ell_deep=(), p_deep=None, double_pass=False) -> Opts:
    """Options of one sign application.  ``ell_deep`` = sizes k_2, k_3, ...
    of the deeper nested levels (Sec. 4.5; k_1 = ell), ``p_deep`` their p
    (None or <= 0: estimated).  ``double_pass``: the low-memory mode of
    Sec. 4.4 (two stored basis vectors, the basis built twice)."""
    o = Opts()
    lib().nks_opts_default(ctypes.byref(o))
    o.k, o.ell, o.tol = int(k), int(ell), float(tol)
    o.precision = _PREC[precision]
    o.p = 0.0 if p is None else float(p)
    o.max_rhi_iter, o.rhi_tol = int(max_rhi_iter), float(rhi_tol)
    o.k_policy, o.ell_policy = int(k_policy), int(ell_policy)
    o.flags = ((FLAG_OVERLAP if overlap else 0) | (FLAG_DEFLATE if deflate else 0)
               | (FLAG_DOUBLE_PASS if double_pass else 0))
    ell_deep = list(ell_deep or ())
    if len(ell_deep) > MAX_LEVELS - 1:
        raise ValueError(f"at most {MAX_LEVELS - 1} deeper levels")
    p_deep = list(p_deep) if p_deep is not None else [None] * len(ell_deep)
    if len(p_deep) != len(ell_deep):
        raise ValueError("p_deep needs one entry per deeper level")
    o.levels = 1 + len(ell_deep)
    for i, (e, q) in enumerate(zip(ell_deep, p_deep)):
        o.ell_deep[i] = int(e)
        o.p_deep[i] = 0.0 if q is None else float(q)
    return o


class Context:
    """One libnks context on the current HIP device."""

    def __init__(self, device: int | None = None):
        torch = _torch()
        self.device = torch.cuda.current_device() if device is None else int(device)
        h = ctypes.c_void_p()
        rc = lib().nks_create(self.device, ctypes.byref(h))
        if rc:
            raise NKSError(rc, "nks_create failed")
        self.h = h
        self._ws = None

    def check(self, rc):
        if rc:
            raise NKSError(rc, lib().nks_last_error(self.h).decode())

    def workspace(self, nbytes: int):
        torch = _torch()
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = None
            self._ws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=f"cuda:{self.device}")
        return self._ws

    def tune_set(self, key: str, value: int):
        self.check(lib().nks_tune_set(self.h, key.encode(), int(value)))

    def tune_get(self, key: str) -> int:
        v = ctypes.c_int()
        self.check(lib().nks_tune_get(self.h, key.encode(), ctypes.byref(v)))
        return v.value

    def profile(self, enable: bool = True):
        """Sample kernel durations with HIP events (see nks_profile_enable)."""
        self.check(lib().nks_profile_enable(self.h, int(bool(enable))))

    def profile_read(self, kernel: str):
        """(timed launches, summed ms, summed algorithmic bytes) for a kernel class."""
        n = ctypes.c_int()
        ms = ctypes.c_double()
        by = ctypes.c_double()
        self.check(lib().nks_profile_read(self.h, KERNEL_CLASSES[kernel], ctypes.byref(n), ctypes.byref(ms),
                                          ctypes.byref(by)))
        return n.value, ms.value, by.value

    def close(self):
        if getattr(self, "h", None):
            self._ws = None
            lib().nks_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Lattice:
    """Gauge links of a dims = (Lx, Ly, Lz, Lt) lattice copied into libnks."""

    def __init__(self, ctx: Context, dims, links, m0: float = 1.6, mu: float = 0.0):
        torch = _torch()
        self.ctx = ctx
        self.dims = tuple(int(d) for d in dims)
        self.V = int(np.prod(self.dims))
        if not isinstance(links, torch.Tensor):
            links = torch.from_numpy(np.ascontiguousarray(links, dtype=np.complex128))
        links = links.to(device=f"cuda:{ctx.device}", dtype=torch.complex128).contiguous()
        if links.numel() != 36 * self.V:
            raise ValueError(f"links must hold 36*V = {36 * self.V} complex numbers, got {links.numel()}")
        d = (ctypes.c_int32 * 4)(*self.dims)
        h = ctypes.c_void_p()
        ctx.check(lib().nks_lattice_create(ctx.h, d, ctypes.c_void_p(links.data_ptr()), ctypes.byref(h)))
        self.h = h
        self.set_params(m0, mu)

    @property
    def n(self):
        return 12 * self.V

    def set_params(self, m0: float, mu: float):
        self.ctx.check(lib().nks_lattice_set_params(self.h, float(m0), float(mu)))
        self.m0, self.mu = float(m0), float(mu)

    def compute_deflation(self, m: int, max_iter: int = 300, tol: float = 1e-10):
        """The m eigenpairs of A with the smallest |lambda|, computed on the GPU
        (left eigenvectors too when mu != 0) and installed for deflate=True jobs
        (see nks_lattice_eigensolve).  Returns (complex eigenvalues ascending in
        |lambda|, residuals, iterations)."""
        lam = np.zeros(2 * m)
        res = np.zeros(m)
        it = ctypes.c_int()
        self.ctx.check(lib().nks_lattice_eigensolve(self.h, int(m), int(max_iter), float(tol),
                                                    lam.ctypes.data_as(_PD), res.ctypes.data_as(_PD),
                                                    ctypes.byref(it)))
        self._defl = None
        return lam[0::2] + 1j * lam[1::2], res, it.value

    def deflation_vectors(self):
        """(r, l): the lattice's deflation eigenvectors as (m, 12*V) complex128
        device tensors in the caller's layout (copies); m = 0 gives empty ones."""
        torch = _torch()
        m = ctypes.c_int()
        self.ctx.check(lib().nks_lattice_get_deflation(self.h, ctypes.byref(m), None, None))
        r = torch.empty((m.value, self.n), dtype=torch.complex128, device=f"cuda:{self.ctx.device}")
        l = torch.empty_like(r)
        if m.value:
            self.ctx.check(lib().nks_lattice_get_deflation(self.h, ctypes.byref(m), ctypes.c_void_p(r.data_ptr()),
                                                           ctypes.c_void_p(l.data_ptr())))
        return r, l

    def set_deflation(self, r, lam, l=None):
        """Eigenpairs for deflate=True jobs: r (and l, default r) of shape
        (m, 12*V) complex128, l_i^H r_j = delta_ij; lam the m eigenvalues."""
        torch = _torch()
        m = 0 if r is None else len(lam)
        if m == 0:
            self.ctx.check(lib().nks_lattice_set_deflation(self.h, 0, None, None, None))
            self._defl = None
            return
        rt = torch.as_tensor(np.ascontiguousarray(r, dtype=np.complex128) if not isinstance(r, torch.Tensor) else r)
        rt = rt.to(device=f"cuda:{self.ctx.device}", dtype=torch.complex128).contiguous()
        lt = None
        if l is not None:
            lt = torch.as_tensor(np.ascontiguousarray(l, dtype=np.complex128) if not isinstance(l, torch.Tensor) else l)
            lt = lt.to(device=f"cuda:{self.ctx.device}", dtype=torch.complex128).contiguous()
        if rt.numel() != m * self.n or (lt is not None and lt.numel() != m * self.n):
            raise ValueError(f"eigenvectors must hold m * 12 * V = {m * self.n} complex numbers")
        la = np.ascontiguousarray(np.asarray(lam, dtype=np.complex128)).view(np.float64)
        self.ctx.check(lib().nks_lattice_set_deflation(self.h, m, ctypes.c_void_p(rt.data_ptr()),
                                                       ctypes.c_void_p(lt.data_ptr()) if lt is not None else None,
                                                       la.ctypes.data_as(_PD)))
        self._defl = (rt, lt)

    def close(self):
        if getattr(self, "h", None):
            lib().nks_lattice_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _vec(lat: Lattice, v):
    torch = _torch()
    if not isinstance(v, torch.Tensor):
        v = torch.from_numpy(np.ascontiguousarray(v, dtype=np.complex128))
    v = v.to(device=f"cuda:{lat.ctx.device}", dtype=torch.complex128).contiguous()
    if v.numel() != lat.n:
        raise ValueError(f"vector must hold 12*V = {lat.n} complex numbers, got {v.numel()}")
    return v


def apply_op(lat: Lattice, v, dagger: bool = False, precision="fp64"):
    """A v (or A^dagger v) with A = gamma5 D_w(mu); returns a new complex128 tensor."""
    torch = _torch()
    v = _vec(lat, v)
    out = torch.empty_like(v)
    lat.ctx.check(lib().nks_apply_op(lat.h, ctypes.c_void_p(v.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                     int(bool(dagger)), _PREC[precision], _stream()))
    return out


def workspace_size(jobs) -> int:
    ctx = jobs[0][0].ctx
    arr, _keep = _job_array(jobs)
    sz = ctypes.c_size_t()
    ctx.check(lib().nks_workspace_size(ctx.h, len(jobs), arr, ctypes.byref(sz)))
    return sz.value


def _job_array(jobs):
    """jobs: list of (lattice, b_tensor, x_tensor, Opts)."""
    arr = (Job * len(jobs))()
    keep = []
    for i, (lat, b, x, o) in enumerate(jobs):
        arr[i].lat = lat.h.value
        arr[i].b = b.data_ptr() if b is not None else None
        arr[i].x = x.data_ptr() if x is not None else None
        arr[i].opts = ctypes.pointer(o)
        keep.append(o)
    return arr, keep


def sign_apply(lat: Lattice, b, k: int = 200, ell: int = 50, p: float | None = None, precision="fp64",
               tol: float = 1e-8, stats: bool = True, out=None, **kw):
    """x ~ sgn(A) b by the nested Krylov-Ritz method; returns (x, stats dict or None)."""
    torch = _torch()
    b = _vec(lat, b)
    x = torch.empty_like(b) if out is None else out
    o = make_opts(k=k, ell=ell, tol=tol, precision=precision, p=p, **kw)
    jobs = [(lat, b, x, o)]
    arr, keep = _job_array(jobs)
    ctx = lat.ctx
    sz = ctypes.c_size_t()
    ctx.check(lib().nks_workspace_size(ctx.h, 1, arr, ctypes.byref(sz)))
    ws = ctx.workspace(sz.value)
    st = Stats()
    ctx.check(lib().nks_sign_apply(ctx.h, lat.h, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                   ctypes.byref(o), ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(),
                                   ctypes.byref(st) if stats else None))
    return x, (st.as_dict() if stats else None)


def sign_apply_noalloc(lat: Lattice, b, k: int = 200, ell: int = 50, p: float | None = None, precision="fp64",
                       tol: float = 1e-8, stats: bool = True, out=None, **kw):
    """sign_apply with the library's static per-GPU workspace (nks_sign_apply_noalloc):
    no device allocation in the call; returns (x, stats dict or None)."""
    torch = _torch()
    b = _vec(lat, b)
    x = torch.empty_like(b) if out is None else out
    o = make_opts(k=k, ell=ell, tol=tol, precision=precision, p=p, **kw)
    st = Stats()
    ctx = lat.ctx
    ctx.check(lib().nks_sign_apply_noalloc(ctx.h, lat.h, ctypes.c_void_p(b.data_ptr()),
                                           ctypes.c_void_p(x.data_ptr()), ctypes.byref(o), _stream(),
                                           ctypes.byref(st) if stats else None))
    return x, (st.as_dict() if stats else None)


def sign_apply_batch(jobs, stats: bool = True, workspace=None):
    """jobs: list of dicts {lat, b, k, ell, p, precision} (or with 'x').

    All jobs run in one call on the current torch stream; jobs on the same
    lattice run in the same stencil launches (each workgroup reads its own
    links).  ``workspace``: a device uint8 tensor
    of at least nks_workspace_size bytes (default: the context's own), so
    that batches can be in flight on several streams at once.  Returns (list
    of x tensors, list of stats dicts or None)."""
    torch = _torch()
    spec = []
    xs = []
    for j in jobs:
        lat = j["lat"]
        b = _vec(lat, j["b"])
        x = j.get("x")
        x = torch.empty_like(b) if x is None else x
        o = make_opts(k=j.get("k", 200), ell=j.get("ell", 50), tol=j.get("tol", 1e-8),
                      precision=j.get("precision", "fp64"), p=j.get("p"),
                      k_policy=j.get("k_policy", POLICY_FIXED), ell_policy=j.get("ell_policy", POLICY_FIXED),
                      overlap=j.get("overlap", False), deflate=j.get("deflate", False),
                      ell_deep=j.get("ell_deep", ()), p_deep=j.get("p_deep"),
                      double_pass=j.get("double_pass", False))
        spec.append((lat, b, x, o))
        xs.append(x)
    ctx = spec[0][0].ctx
    arr, keep = _job_array(spec)
    sz = ctypes.c_size_t()
    ctx.check(lib().nks_workspace_size(ctx.h, len(spec), arr, ctypes.byref(sz)))
    if workspace is None:
        ws = ctx.workspace(sz.value)
    else:
        ws = workspace
        if ws.dtype != torch.uint8 or not ws.is_cuda or ws.numel() < sz.value:
            raise ValueError(f"workspace must be a device uint8 tensor of >= {sz.value} bytes")
    sts = (Stats * len(spec))()
    ctx.check(lib().nks_sign_apply_batch(ctx.h, len(spec), arr, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                         _stream(), sts if stats else None))
    return xs, ([s.as_dict() for s in sts] if stats else None)


def overlap_apply(lat: Lattice, b, **kw):
    """D_ov(mu) b = b + gamma5 sgn(gamma5 D_w(mu)) b (Sec. 2); same options as sign_apply."""
    return sign_apply(lat, b, overlap=True, **kw)


def outer_basis(lat: Lattice, b, k: int, precision="fp64"):
    """Steps 1-2 only: returns (alpha, beta, gamma) as complex numpy arrays and stats."""
    b = _vec(lat, b)
    o = make_opts(k=k, ell=2, precision=precision)
    jobs = [(lat, b, None, o)]
    arr, keep = _job_array(jobs)
    ctx = lat.ctx
    sz = ctypes.c_size_t()
    ctx.check(lib().nks_workspace_size(ctx.h, 1, arr, ctypes.byref(sz)))
    ws = ctx.workspace(sz.value)
    kk = o.k + (o.k & 1)
    a = np.zeros(2 * kk)
    bb = np.zeros(2 * max(kk - 1, 1))
    g = np.zeros(2 * max(kk - 1, 1))
    st = Stats()
    P = lambda arr_: arr_.ctypes.data_as(_PD)  # noqa: E731
    ctx.check(lib().nks_outer_basis(ctx.h, lat.h, ctypes.c_void_p(b.data_ptr()), ctypes.byref(o),
                                    ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(), P(a), P(bb), P(g),
                                    ctypes.byref(st)))
    ku = st.k_used
    a = a.view(np.complex128)[:ku]
    bb = bb.view(np.complex128)[:max(ku - 1, 0)]
    g = g.view(np.complex128)[:max(ku - 1, 0)]
    return a, bb, g, st.as_dict()


MLP_NPARAMS = 5378
POLICY_NFEAT = 16
POLICY_NFLOATS = MLP_NPARAMS + 2 * POLICY_NFEAT + 4
LEARN_K0 = 100
LABEL_NK, LABEL_NELL, LABEL_DK = 60, 4, 20
LABEL_WORDS = POLICY_NFEAT + LABEL_NK * (1 + LABEL_NELL)


def policy_load(ctx: Context, blob):
    """Load the learned-policy network (float32 vector of POLICY_NFLOATS:
    parameters, feature mean/scale, target mean/scale) for later calls."""
    blob = np.ascontiguousarray(blob, dtype=np.float32).ravel()
    ctx.check(lib().nks_policy_load(ctx.h, blob.ctypes.data, int(blob.size)))


def load_policy(ctx: Context, path: str | None = None) -> dict:
    """Load the trained network shipped with the package (or the file at
    path, written by ``python -m paper_0912_4457_amd.policy``); returns its
    training metadata."""
    from . import policy as _p
    blob, meta = _p.load(path or _p.DEFAULT_PATH)
    policy_load(ctx, blob)
    return meta


def policy_label(jobs):
    """Training labels for the learned policy; jobs: list of dicts {lat, b, k,
    ell, tol, precision}.  Returns a (njobs, LABEL_WORDS) float64 array laid
    out as documented for nks_policy_label."""
    spec = []
    for j in jobs:
        lat = j["lat"]
        o = make_opts(k=j.get("k", 600), ell=j.get("ell", 256), tol=j.get("tol", 1e-8),
                      precision=j.get("precision", "fp64"))
        spec.append((lat, _vec(lat, j["b"]), None, o))
    ctx = spec[0][0].ctx
    arr, keep = _job_array(spec)
    out = np.zeros((len(spec), LABEL_WORDS))
    ctx.check(lib().nks_policy_label(ctx.h, len(spec), arr, out.ctypes.data_as(_PD)))
    return out


def _f32(t):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        t = torch.from_numpy(np.ascontiguousarray(t, dtype=np.float32))
    return t.to(device="cuda", dtype=torch.float32).contiguous()


def mlp_forward(ctx: Context, params, x):
    """y = MLP(x) for x of shape (batch, 16); params: float32 vector of 5378."""
    torch = _torch()
    params, x = _f32(params), _f32(x)
    y = torch.empty((x.shape[0], 2), dtype=torch.float32, device=x.device)
    ctx.check(lib().nks_mlp_forward(ctx.h, params.data_ptr(), x.data_ptr(), x.shape[0], y.data_ptr(), _stream()))
    return y


def mlp_backward(ctx: Context, params, x, t):
    """(loss, grad) of 0.5 * mean ||MLP(x) - t||^2."""
    torch = _torch()
    params, x, t = _f32(params), _f32(x), _f32(t)
    g = torch.empty(MLP_NPARAMS, dtype=torch.float32, device=x.device)
    loss = torch.empty(1, dtype=torch.float32, device=x.device)
    ctx.check(lib().nks_mlp_backward(ctx.h, params.data_ptr(), x.data_ptr(), t.data_ptr(), x.shape[0], g.data_ptr(),
                                     loss.data_ptr(), _stream()))
    return loss, g


def mlp_adam_step(ctx: Context, params, grad, m, v, step: int, lr: float):
    """In-place Adam update of the float32 tensors params, m, v."""
    ctx.check(lib().nks_mlp_adam_step(ctx.h, params.data_ptr(), grad.data_ptr(), m.data_ptr(), v.data_ptr(),
                                      int(step), float(lr), _stream()))


def nested_step(ctx: Context, alpha, beta, gamma, hermitian: bool, ell: int, p: float | None = None,
                max_rhi_iter: int = 50, rhi_tol: float = 1e-14, ell_policy: int = POLICY_FIXED,
                tol: float = 1e-8, ell_deep=(), p_deep=None):
    """Steps 3-5 on a given tridiagonal H_k: returns (c ~ sgn(H_k) e_1, stats).

    With ell_policy=POLICY_DOUBLING, ``ell`` is the largest inner size allowed."""
    alpha = np.ascontiguousarray(alpha, dtype=np.complex128)
    k = alpha.size
    beta = np.ascontiguousarray(beta if k > 1 else np.zeros(1), dtype=np.complex128)
    gamma = np.ascontiguousarray(gamma if k > 1 else np.zeros(1), dtype=np.complex128)
    o = make_opts(k=k, ell=ell, p=p, max_rhi_iter=max_rhi_iter, rhi_tol=rhi_tol, ell_policy=ell_policy, tol=tol,
                  ell_deep=ell_deep, p_deep=p_deep)
    c = np.zeros(k, dtype=np.complex128)
    st = Stats()
    P = lambda arr_: arr_.view(np.float64).ctypes.data_as(_PD)  # noqa: E731
    ctx.check(lib().nks_nested_step(ctx.h, k, P(alpha), P(beta), P(gamma), int(bool(hermitian)), ctypes.byref(o),
                                    P(c), ctypes.byref(st)))
    return c, st.as_dict()
