"""ctypes binding of libifctn.so (include/ifctn.h).

Argument marshalling only: every step of the completion runs in the HIP
library.  The functions keep the C names; :class:`Job` is a small convenience
wrapper that takes torch tensors (torch provides device memory and streams).
The library must be built (``__graft_entry__.build()``); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

try:  # load torch's HIP runtime first so that the library shares it
    import torch
except Exception:  # pragma: no cover - torch is part of the image
    torch = None

from . import workloads

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libifctn.so")

IFCTN_MAX_ORDER = 5
IFCTN_MAX_RANK = 36
IFCTN_OK, IFCTN_E_INVAL, IFCTN_E_NOMEM, IFCTN_E_HIP, IFCTN_E_STATE, IFCTN_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
IFCTN_FP32, IFCTN_BF16_REFINE, IFCTN_FP64 = 0, 1, 2
KC_CONTRACT, KC_SOLVE, KC_UPDATE, KC_GRAM, KC_UROW = 0, 1, 2, 3, 4

EXPORTED = [
    "ifctn_num_factor_entries", "ifctn_workspace_bytes", "ifctn_init", "ifctn_sweep",
    "ifctn_reconstruct", "ifctn_get_factors", "ifctn_destroy", "ifctn_complete",
    "ifctn_assemble", "ifctn_timing_enable", "ifctn_timing_query", "ifctn_last_error",
    "ifctn_promote", "ifctn_server_create", "ifctn_server_submit", "ifctn_server_poll",
    "ifctn_server_queued", "ifctn_server_destroy", "ifctn_set_option", "ifctn_image_metrics",
    "ifctn_plan_blocks", "ifctn_assemble_noalloc", "ifctn_default_factors",
]


class IfctnBlockPlan(ctypes.Structure):
    _fields_ = [("route", ctypes.c_int32), ("reserved", ctypes.c_int32), ("gamma_fma", ctypes.c_double)]


class IfctnParams(ctypes.Structure):
    _fields_ = [
        ("order", ctypes.c_int32),
        ("dims", ctypes.c_int64 * IFCTN_MAX_ORDER),
        ("ranks", (ctypes.c_int32 * IFCTN_MAX_ORDER) * IFCTN_MAX_ORDER),
        ("rho", ctypes.c_double),
        ("rho_x", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("refine_sweeps", ctypes.c_int32),
    ]


class IfctnStats(ctypes.Structure):
    _fields_ = [
        ("rel_change", ctypes.c_double),
        ("objective", ctypes.c_double),
        ("x_norm2", ctypes.c_double),
        ("dx_norm2", ctypes.c_double),
        ("dg_norm2", ctypes.c_double),
        ("sweeps_done", ctypes.c_int32),
        ("converged", ctypes.c_int32),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class IfctnServerConfig(ctypes.Structure):
    _fields_ = [
        ("hbm_budget_bytes", ctypes.c_size_t),
        ("max_active", ctypes.c_int32),
        ("num_streams", ctypes.c_int32),
        ("sweeps_per_round", ctypes.c_int32),
        ("device", ctypes.c_int32),
    ]


class IfctnRequest(ctypes.Structure):
    _fields_ = [
        ("params", IfctnParams),
        ("O_dev", ctypes.c_void_p),
        ("mask_dev", ctypes.c_void_p),
        ("G0_host", ctypes.POINTER(ctypes.c_double)),
        ("t_max", ctypes.c_int32),
        ("eps", ctypes.c_double),
        ("X_out_dev", ctypes.c_void_p),
        ("tag", ctypes.c_uint64),
    ]


class IfctnCompletion(ctypes.Structure):
    _fields_ = [
        ("tag", ctypes.c_uint64),
        ("status", ctypes.c_int32),
        ("stats", IfctnStats),
        ("t_submit", ctypes.c_double),
        ("t_admit", ctypes.c_double),
        ("t_done", ctypes.c_double),
    ]


class IfctnError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"ifctn status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libifctn.so (once) and declare the C signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    P, S = ctypes.POINTER(IfctnParams), ctypes.POINTER(IfctnStats)
    vp, dp, i32, st = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int32, ctypes.c_int
    sig = {
        "ifctn_num_factor_entries": (ctypes.c_size_t, [P]),
        "ifctn_workspace_bytes": (ctypes.c_size_t, [P]),
        "ifctn_init": (st, [P, vp, vp, dp, vp, ctypes.POINTER(vp)]),
        "ifctn_sweep": (st, [vp, i32, S]),
        "ifctn_reconstruct": (st, [vp, vp, i32]),
        "ifctn_get_factors": (st, [vp, dp]),
        "ifctn_destroy": (st, [vp]),
        "ifctn_complete": (st, [P, vp, vp, dp, i32, ctypes.c_double, vp, S, vp]),
        "ifctn_assemble": (st, [P, dp, vp, vp]),
        "ifctn_assemble_noalloc": (st, [P, dp, vp, vp]),
        "ifctn_default_factors": (st, [P, vp, vp, ctypes.c_uint64, vp, dp]),
        "ifctn_timing_enable": (st, [vp, i32]),
        "ifctn_timing_query": (st, [vp, i32, dp, ctypes.POINTER(ctypes.c_int64)]),
        "ifctn_last_error": (ctypes.c_char_p, []),
        "ifctn_promote": (st, [vp]),
        "ifctn_server_create": (st, [ctypes.POINTER(IfctnServerConfig), ctypes.POINTER(vp)]),
        "ifctn_server_submit": (st, [vp, ctypes.POINTER(IfctnRequest)]),
        "ifctn_server_poll": (st, [vp, ctypes.POINTER(IfctnCompletion), i32, ctypes.POINTER(i32), i32]),
        "ifctn_server_queued": (st, [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        "ifctn_server_destroy": (st, [vp]),
        "ifctn_set_option": (st, [ctypes.c_char_p, ctypes.c_int64]),
        "ifctn_plan_blocks": (st, [P, ctypes.POINTER(IfctnBlockPlan)]),
        "ifctn_image_metrics": (st, [vp, vp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, i32, ctypes.c_double,
                                     dp, dp, dp, dp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(status):
    if status != IFCTN_OK:
        raise IfctnError(status, lib().ifctn_last_error().decode())


def make_params(dims, ranks, rho=0.1, rho_x=0.0, precision=IFCTN_FP32, refine_sweeps=0) -> IfctnParams:
    p = IfctnParams()
    p.order = len(dims)
    for m, d in enumerate(dims):
        p.dims[m] = int(d)
    for a in range(len(dims)):
        for b in range(len(dims)):
            p.ranks[a][b] = int(ranks[a][b]) if a != b else 0
    p.rho, p.rho_x, p.precision, p.refine_sweeps = float(rho), float(rho_x), int(precision), int(refine_sweeps)
    return p


def set_option(name: str, value: int):
    """Process-wide tuning option (ifctn_set_option); value < 0 = default."""
    _check(lib().ifctn_set_option(name.encode(), int(value)))


def _dptr(arr: np.ndarray):
    return arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def num_factor_entries(dims, ranks) -> int:
    return int(lib().ifctn_num_factor_entries(ctypes.byref(make_params(dims, ranks))))


ROUTE_PERCOLUMN, ROUTE_PHASED, ROUTE_GAMMA, ROUTE_LARGE = 0, 1, 2, 3


def plan_blocks(dims, ranks, precision=IFCTN_FP32):
    """Per mode k: (route, multiply-adds of building Gamma_k) (ifctn_plan_blocks)."""
    out = (IfctnBlockPlan * IFCTN_MAX_ORDER)()
    _check(lib().ifctn_plan_blocks(ctypes.byref(make_params(tuple(dims), ranks, precision=precision)), out))
    return [(int(out[k].route), float(out[k].gamma_fma)) for k in range(len(dims))]


def workspace_bytes(dims, ranks, precision=IFCTN_FP32) -> int:
    return int(lib().ifctn_workspace_bytes(ctypes.byref(make_params(dims, ranks, precision=precision))))


def _stream_handle():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dtype(precision):
    return torch.float64 if precision == IFCTN_FP64 else torch.float32


class Job:
    """A completion job on the current torch device and stream."""

    def __init__(self, O, mask, G0, dims, ranks, rho=0.1, rho_x=0.0, precision=IFCTN_FP32):
        self.dims = tuple(int(d) for d in dims)
        self.ranks = np.asarray(ranks)
        self.precision = precision
        self.params = make_params(self.dims, self.ranks, rho, rho_x, precision)
        dt = _dtype(precision)
        self.O = torch.as_tensor(np.asarray(O)).to(device="cuda", dtype=dt).contiguous()
        self.mask = torch.as_tensor(np.asarray(mask, dtype=np.uint8)).to("cuda").contiguous()
        # G0 None: the library's seeded default (ifctn_default_factors, seed 0)
        if G0 is None:
            self._g0 = None
        else:
            g0 = G0 if isinstance(G0, np.ndarray) and G0.ndim == 1 else workloads.pack(G0, self.dims, self.ranks)
            self._g0 = np.ascontiguousarray(g0, dtype=np.float64)
        h = ctypes.c_void_p()
        _check(lib().ifctn_init(ctypes.byref(self.params), ctypes.c_void_p(self.O.data_ptr()),
                                ctypes.c_void_p(self.mask.data_ptr()),
                                None if self._g0 is None else _dptr(self._g0),
                                _stream_handle(), ctypes.byref(h)))
        self.handle = h

    def sweep(self, n=1, stats=True):
        s = IfctnStats()
        _check(lib().ifctn_sweep(self.handle, int(n), ctypes.byref(s) if stats else None))
        return s.as_dict() if stats else None

    def reconstruct(self, which=0):
        out = torch.empty(self.dims, dtype=_dtype(self.precision), device="cuda")
        _check(lib().ifctn_reconstruct(self.handle, ctypes.c_void_p(out.data_ptr()), int(which)))
        return out

    def x(self):
        return self.reconstruct(1)

    def xhat(self):
        return self.reconstruct(0)

    def factors(self):
        n = num_factor_entries(self.dims, self.ranks)
        buf = np.empty(n, dtype=np.float64)
        _check(lib().ifctn_get_factors(self.handle, _dptr(buf)))
        return workloads.unpack(buf, self.dims, self.ranks)

    def promote(self):
        """End the bfloat16 phase of a BF16_REFINE job (later sweeps stream float32)."""
        _check(lib().ifctn_promote(self.handle))

    def timing(self, enable: bool):
        _check(lib().ifctn_timing_enable(self.handle, 1 if enable else 0))

    def timing_query(self, kernel_class):
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _check(lib().ifctn_timing_query(self.handle, int(kernel_class), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def close(self):
        if getattr(self, "handle", None):
            lib().ifctn_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def complete(O, mask, G0, dims, ranks, t_max, eps=0.0, rho=0.1, precision=IFCTN_FP32, refine_sweeps=0):
    """Algorithm 1 end to end through ifctn_complete; returns (X, stats)."""
    dims = tuple(int(d) for d in dims)
    params = make_params(dims, ranks, rho, 0.0, precision, refine_sweeps)
    dt = _dtype(precision)
    if isinstance(O, torch.Tensor):
        Ot = O.to(device="cuda", dtype=dt).contiguous()
    else:
        Ot = torch.as_tensor(np.asarray(O)).to(device="cuda", dtype=dt).contiguous()
    if isinstance(mask, torch.Tensor):
        Mt = mask.to(device="cuda", dtype=torch.uint8).contiguous()
    else:
        Mt = torch.as_tensor(np.asarray(mask, dtype=np.uint8)).to("cuda").contiguous()
    g0 = None if G0 is None else np.ascontiguousarray(
        workloads.pack(G0, dims, ranks) if isinstance(G0, dict) else G0, dtype=np.float64)
    out = torch.empty(dims, dtype=dt, device="cuda")
    s = IfctnStats()
    _check(lib().ifctn_complete(ctypes.byref(params), ctypes.c_void_p(Ot.data_ptr()),
                                ctypes.c_void_p(Mt.data_ptr()), None if g0 is None else _dptr(g0),
                                int(t_max), float(eps),
                                ctypes.c_void_p(out.data_ptr()), ctypes.byref(s), _stream_handle()))
    return out, s.as_dict()


def default_factors(O, mask, dims, ranks, seed=0, precision=IFCTN_FP32, packed=False):
    """The library's seeded default G^0 (ifctn_default_factors): uniform
    entries scaled so that iFCTN(G^0) has the observed entries' root mean
    square as its expected value.  A dict {(k, i): R_ki x I_k}, or the packed
    float64 array with packed=True."""
    dims = tuple(int(d) for d in dims)
    params = make_params(dims, ranks, precision=precision)
    dt = _dtype(precision)
    Ot = torch.as_tensor(np.asarray(O) if not isinstance(O, torch.Tensor) else O).to(device="cuda", dtype=dt)
    Ot = Ot.contiguous()
    Mt = torch.as_tensor(np.asarray(mask, dtype=np.uint8) if not isinstance(mask, torch.Tensor) else mask)
    Mt = Mt.to(device="cuda", dtype=torch.uint8).contiguous()
    buf = np.empty(num_factor_entries(dims, ranks), dtype=np.float64)
    _check(lib().ifctn_default_factors(ctypes.byref(params), ctypes.c_void_p(Ot.data_ptr()),
                                       ctypes.c_void_p(Mt.data_ptr()), ctypes.c_uint64(int(seed)),
                                       _stream_handle(), _dptr(buf)))
    return buf if packed else workloads.unpack(buf, dims, ranks)


def assemble(dims, ranks, G, precision=IFCTN_FP32, out=None, noalloc=False):
    """iFCTN(G) materialised on the GPU by the library (eq. (iFCTN)).

    out: an existing contiguous CUDA tensor of shape dims and the precision's
    dtype to write into (a new one otherwise).  noalloc: call
    ifctn_assemble_noalloc, which stages factors and edge matrices in the
    library's fixed per-GPU array instead of allocating device memory."""
    dims = tuple(int(d) for d in dims)
    params = make_params(dims, ranks, precision=precision)
    g = np.ascontiguousarray(workloads.pack(G, dims, ranks) if isinstance(G, dict) else G, dtype=np.float64)
    if out is None:
        out = torch.empty(dims, dtype=_dtype(precision), device="cuda")
    elif (tuple(out.shape) != dims or out.dtype != _dtype(precision) or not out.is_cuda
          or not out.is_contiguous()):
        raise ValueError("out must be a contiguous CUDA tensor of shape %s and dtype %s"
                         % (dims, _dtype(precision)))
    fn = lib().ifctn_assemble_noalloc if noalloc else lib().ifctn_assemble
    _check(fn(ctypes.byref(params), _dptr(g), ctypes.c_void_p(out.data_ptr()), _stream_handle()))
    return out


class Server:
    """Continuous-batching server (ifctn_server_*): requests are admitted by
    slots and HBM budget and overlap on the device.  Inputs are torch CUDA
    tensors (or numpy arrays, copied to the device); the binding keeps them
    and the output tensor alive until the completion is polled."""

    def __init__(self, hbm_budget_bytes, max_active=8, num_streams=8, sweeps_per_round=10, device=None):
        cfg = IfctnServerConfig()
        cfg.hbm_budget_bytes = int(hbm_budget_bytes)
        cfg.max_active, cfg.num_streams = int(max_active), int(num_streams)
        cfg.sweeps_per_round = int(sweeps_per_round)
        cfg.device = int(torch.cuda.current_device() if device is None else device)
        h = ctypes.c_void_p()
        _check(lib().ifctn_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self.handle = h
        self._live = {}
        self._next = 0

    def submit(self, O, mask, G0, dims, ranks, t_max, eps=0.0, rho=0.1, precision=IFCTN_FP32, refine_sweeps=0,
               tag=None, sync=True):
        dims = tuple(int(d) for d in dims)
        params = make_params(dims, ranks, rho, 0.0, precision, refine_sweeps)
        dt = _dtype(precision)
        Ot = torch.as_tensor(O).to(device="cuda", dtype=dt).contiguous()
        Mt = torch.as_tensor(np.asarray(mask, dtype=np.uint8) if isinstance(mask, np.ndarray) else mask)
        Mt = Mt.to(device="cuda", dtype=torch.uint8).contiguous()
        if G0 is None:   # the library's seeded default (seed 0), drawn now on the current stream
            g0 = default_factors(Ot, Mt, dims, ranks, seed=0, precision=precision, packed=True)
        else:
            g0 = np.ascontiguousarray(workloads.pack(G0, dims, ranks) if isinstance(G0, dict) else G0,
                                      dtype=np.float64)
        out = torch.empty(dims, dtype=dt, device="cuda")
        if tag is None:
            tag = self._next
        self._next = max(self._next, int(tag)) + 1
        if sync:  # the server's streams do not wait for torch's
            torch.cuda.current_stream().synchronize()
        r = IfctnRequest()
        r.params = params
        r.O_dev, r.mask_dev = Ot.data_ptr(), Mt.data_ptr()
        r.G0_host = _dptr(g0)
        r.t_max, r.eps = int(t_max), float(eps)
        r.X_out_dev = out.data_ptr()
        r.tag = int(tag)
        _check(lib().ifctn_server_submit(self.handle, ctypes.byref(r)))
        self._live[int(tag)] = (Ot, Mt, out)
        return int(tag)

    def poll(self, max_n=64, wait_ms=0):
        buf = (IfctnCompletion * max_n)()
        n = ctypes.c_int32()
        _check(lib().ifctn_server_poll(self.handle, buf, int(max_n), ctypes.byref(n), int(wait_ms)))
        res = []
        for q in range(n.value):
            c = buf[q]
            keep = self._live.pop(int(c.tag), None)
            res.append({"tag": int(c.tag), "status": int(c.status), "stats": c.stats.as_dict(),
                        "t_submit": c.t_submit, "t_admit": c.t_admit, "t_done": c.t_done,
                        "X": keep[2] if keep else None})
        return res

    def queued(self):
        a, b = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().ifctn_server_queued(self.handle, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def close(self):
        if getattr(self, "handle", None):
            lib().ifctn_server_destroy(self.handle)
            self.handle = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def image_metrics(X, ref, peak=1.0):
    """MPSNR and MSSIM (ifctn_image_metrics) of an H x W x B tensor against a
    reference; returns (mpsnr, mssim, psnr_per_band, ssim_per_band)."""
    Xt = torch.as_tensor(X)
    dt = torch.float64 if Xt.dtype == torch.float64 else torch.float32
    Xt = Xt.to(device="cuda", dtype=dt).contiguous()
    Rt = torch.as_tensor(ref).to(device="cuda", dtype=dt).contiguous()
    if Xt.dim() != 3 or Xt.shape != Rt.shape:
        raise ValueError("image_metrics needs two H x W x B tensors of the same shape")
    H, Wd, B = (int(x) for x in Xt.shape)
    ps = np.empty(B)
    ss = np.empty(B)
    mp, ms = ctypes.c_double(), ctypes.c_double()
    _check(lib().ifctn_image_metrics(ctypes.c_void_p(Xt.data_ptr()), ctypes.c_void_p(Rt.data_ptr()), H, Wd, B,
                                     IFCTN_FP64 if dt == torch.float64 else IFCTN_FP32, float(peak), _dptr(ps),
                                     _dptr(ss), ctypes.byref(mp), ctypes.byref(ms), _stream_handle()))
    return mp.value, ms.value, ps, ss

