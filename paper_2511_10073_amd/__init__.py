"""Python binding of libahr, the MI355X signed netlist graph filter.

Argument marshalling only: every step runs in the HIP library.  PyTorch
provides device memory and the current stream.  The library must have been
built (``paper_2511_10073_amd.build``); importing it without ``libahr.so``
raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libahr.so")

FIXED = 1
MACRO = 2
EXPAND_MACRO_PINS = 1
MACRO_HINTS = 2
BIN_HINTS = 4
ALL_HINTS = 7
LAYOUT_AUTO = 8             # netlist order where the placement's Hilbert order has no locality
LAYOUT_NETLIST = 16         # the Cuthill-McKee order of the netlist
HOP_ROW_BLOCK = 256       # lanes_per_row value selecting the row-block hop
HOP_AUTO = 1024           # lanes_per_row value: the shape follows each graph's execution order
LAMBDA_GERSHGORIN = 0
LAMBDA_FIXED = 1

OK, EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED = 0, -1, -2, -3, -4


class AhrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ahr error {code}: {msg}")
        self.code = code


class _Netlist(ctypes.Structure):
    _fields_ = [("n_inst", ctypes.c_int32), ("n_nets", ctypes.c_int32), ("n_pins", ctypes.c_int32),
                ("reserved0", ctypes.c_int32), ("net_ptr", ctypes.c_void_p), ("pin_node", ctypes.c_void_p),
                ("pin_off", ctypes.c_void_p), ("net_w", ctypes.c_void_p), ("node_flags", ctypes.c_void_p),
                ("node_size", ctypes.c_void_p), ("die", ctypes.c_float * 4)]


class _HintParams(ctypes.Structure):
    _fields_ = [("nbx", ctypes.c_int32), ("nby", ctypes.c_int32), ("detection_ratio", ctypes.c_float),
                ("bin_capacity", ctypes.c_float), ("mu", ctypes.c_float), ("clique_max", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("prune_tau", ctypes.c_float)]


class _FilterSpec(ctypes.Structure):
    _fields_ = [("nbands", ctypes.c_int32), ("k", ctypes.c_int32 * 4), ("alpha", ctypes.c_float * 4),
                ("sigma", ctypes.c_float), ("lambda_mode", ctypes.c_int32), ("lambda_fixed", ctypes.c_float)]


class _GiftSpec(ctypes.Structure):
    _fields_ = [("nbands", ctypes.c_int32), ("k", ctypes.c_int32 * 4), ("alpha", ctypes.c_float * 4),
                ("sigma", ctypes.c_float * 4)]


class _ChargeParams(ctypes.Structure):
    _fields_ = ([(n, ctypes.c_int32) for n in ("model", "t", "T", "nbx", "nby")]
                + [(n, ctypes.c_float) for n in ("sigma_factor", "k_factor", "r0", "r1", "beta_min", "beta_max",
                                                 "alpha0", "alpha1")])


CHARGE_GAUSSIAN, CHARGE_EXP, CHARGE_LINEAR, CHARGE_SIGMOID = 0, 1, 2, 3


def charge_params(model=CHARGE_EXP, t=0, T=300, nbx=32, nby=32, sigma_factor=0.005, k_factor=1.0, r0=1e-3, r1=0.9,
                  beta_min=0.1, beta_max=1.0, alpha0=0.2, alpha1=0.8):
    return _ChargeParams(model, t, T, nbx, nby, sigma_factor, k_factor, r0, r1, beta_min, beta_max, alpha0, alpha1)


def charge_schedule(cp) -> float:
    v = ctypes.c_double()
    _check(load().ahr_charge_schedule(ctypes.byref(cp), ctypes.byref(v)))
    return v.value


def macro_charge(netlist, g, cp, out=None, stream=None):
    """Per-bin macro charge masses (device float64 [nby * nbx])."""
    if out is None:
        out = torch.empty(cp.nbx * cp.nby, dtype=torch.float64, device=g.device)
    _check(load().ahr_macro_charge(ctypes.byref(netlist.c), _ptr(g), g.shape[1], ctypes.byref(cp), _ptr(out),
                                   _stream(stream)))
    return out


class _GraphInfo(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in (
        "n_inst", "n_tot", "first_mpin", "first_star", "first_mvirt", "first_bvirt", "nnz_net", "nnz_hint",
        "n_hint_cells", "n_long_rows", "hint_version", "layout", "hop_lanes", "reserved")] + [
            ("ws_bytes", ctypes.c_int64),
                                                                        ("ws_peak", ctypes.c_int64)]


class _GraphHost(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in (
        "net_row_ptr", "net_col", "net_q", "hint_row_ptr", "hint_col", "hint_val", "degree", "scale", "lambda_up")]


class _BatchInfo(ctypes.Structure):
    _fields_ = ([(n, ctypes.c_int32) for n in ("n_graphs", "n_inst", "n_tot", "n_long_rows")]
                + [(n, ctypes.c_int64) for n in ("nnz_net", "nnz_hint")]
                + [(n, ctypes.c_int32) for n in ("n_captured", "reserved")])


class _Profile(ctypes.Structure):
    _fields_ = ([(n, ctypes.c_double) for n in ("build_ms", "hints_ms", "norm_ms", "expand_ms", "hop_ms",
                                                 "relax_ms", "hpwl_ms")]
                + [(n, ctypes.c_int64) for n in ("build_calls", "hints_calls", "norm_calls", "expand_calls",
                                                  "hop_launches", "relax_calls", "hpwl_calls")]
                + [("hop_bytes", ctypes.c_double), ("mlp_ms", ctypes.c_double), ("mlp_calls", ctypes.c_int64),
                   ("wa_ms", ctypes.c_double), ("wa_calls", ctypes.c_int64), ("wa_bytes", ctypes.c_double)])


class _Mlp(ctypes.Structure):
    _fields_ = [("params", ctypes.c_void_p), ("beta", ctypes.c_float * 4), ("validated", ctypes.c_int32)]


MLP_NPARAM = 4801
MLP_FEATURE_STRIDE = 8


_lib = None


def load() -> ctypes.CDLL:
    """Load libahr.so (built in-tree); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run paper_2511_10073_amd.build.build() first")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32 = ctypes.c_void_p, ctypes.c_int32
    lib.ahr_last_error.restype = ctypes.c_char_p
    lib.ahr_version.restype = ctypes.c_char_p
    sigs = {
        "ahr_graph_build": [ctypes.POINTER(_Netlist), ctypes.POINTER(_HintParams), vp, i32, vp, ctypes.c_size_t, vp,
                            ctypes.POINTER(vp)],
        "ahr_graph_workspace_size": [ctypes.POINTER(_Netlist), ctypes.POINTER(_HintParams), i32, vp,
                                     ctypes.POINTER(ctypes.c_size_t)],
        "ahr_graph_update_hints": [vp, vp, i32, vp],
        "ahr_graph_get_info": [vp, ctypes.POINTER(_GraphInfo)],
        "ahr_graph_export": [vp, ctypes.POINTER(_GraphHost), vp],
        "ahr_filter": [vp, ctypes.POINTER(_FilterSpec), vp, vp, i32, vp],
        "ahr_gift": [vp, ctypes.POINTER(_GiftSpec), vp, vp, i32, vp],
        "ahr_graph_refine": [vp, ctypes.POINTER(_FilterSpec), vp, i32, i32, ctypes.c_float, vp, vp],
        "ahr_refine": [ctypes.POINTER(_Netlist), ctypes.POINTER(_HintParams), ctypes.POINTER(_FilterSpec), vp, i32, i32,
                       ctypes.c_float, vp, vp, ctypes.c_size_t, vp],
        "ahr_hpwl": [ctypes.POINTER(_Netlist), vp, i32, vp, vp],
        "ahr_hpwl_noalloc": [ctypes.POINTER(_Netlist), vp, i32, vp, vp],
        "ahr_wl_create": [ctypes.POINTER(_Netlist), vp, ctypes.POINTER(vp)],
        "ahr_charge_schedule": [ctypes.POINTER(_ChargeParams), ctypes.POINTER(ctypes.c_double)],
        "ahr_macro_charge": [ctypes.POINTER(_Netlist), vp, i32, ctypes.POINTER(_ChargeParams), vp, vp],
        "ahr_wa": [vp, vp, i32, ctypes.c_float, vp, vp, vp],
        "ahr_filter_learned": [vp, ctypes.POINTER(_FilterSpec), ctypes.POINTER(_Mlp), vp, vp, i32,
                               ctypes.POINTER(i32), vp],
        "ahr_filter_features": [vp, ctypes.POINTER(_FilterSpec), vp, i32, vp, vp, vp, vp],
        "ahr_refine_learned": [vp, ctypes.POINTER(_FilterSpec), ctypes.POINTER(_Mlp), vp, i32, i32, ctypes.c_float, vp,
                               ctypes.POINTER(i32), vp],
        "ahr_mlp_forward": [vp, vp, ctypes.c_int64, vp, vp],
        "ahr_mlp_loss_grad": [vp, vp, vp, ctypes.c_int64, vp, vp, i32, vp],
        "ahr_mlp_adam": [vp, vp, vp, vp, i32, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, vp],
        "ahr_batch_build": [vp, vp, i32, vp, i32, vp, ctypes.POINTER(vp)],
        "ahr_batch_get_info": [vp, ctypes.POINTER(_BatchInfo)],
        "ahr_batch_filter": [vp, ctypes.POINTER(_FilterSpec), vp, vp, i32, i32, vp],
        "ahr_batch_set_config": [vp, i32, i32, i32],
        "ahr_batch_get_config": [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)],
        "ahr_batch_autotune": [vp, ctypes.POINTER(_FilterSpec), i32, vp, ctypes.POINTER(i32), ctypes.POINTER(i32),
                               ctypes.POINTER(ctypes.c_float)],
    }
    for name, args in sigs.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int32
    lib.ahr_filter_tune.argtypes = [i32, i32]
    lib.ahr_filter_tune.restype = ctypes.c_int32
    lib.ahr_filter_get_tune.argtypes = [ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.ahr_filter_get_tune.restype = ctypes.c_int32
    lib.ahr_profile_enable.argtypes = [i32]
    lib.ahr_profile_enable.restype = ctypes.c_int32
    lib.ahr_profile_read.argtypes = [ctypes.POINTER(_Profile), i32]
    lib.ahr_profile_read.restype = ctypes.c_int32
    lib.ahr_hpwl_noalloc_bytes.argtypes = []
    lib.ahr_hpwl_noalloc_bytes.restype = ctypes.c_size_t
    lib.ahr_wl_destroy.argtypes = [vp]
    lib.ahr_wl_destroy.restype = None
    lib.ahr_graph_destroy.argtypes = [vp]
    lib.ahr_graph_destroy.restype = None
    lib.ahr_batch_destroy.argtypes = [vp]
    lib.ahr_batch_destroy.restype = None
    _lib = lib
    return lib


def _check(code):
    if code != OK:
        raise AhrError(code, load().ahr_last_error().decode())


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def filter_tune(lanes_per_row: int = 0, nontemporal: int = -1):
    """Set the hop launch shape (0 / -1 keep the current values)."""
    _check(load().ahr_filter_tune(lanes_per_row, nontemporal))


def filter_get_tune() -> tuple:
    a, b = ctypes.c_int32(), ctypes.c_int32()
    _check(load().ahr_filter_get_tune(ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def profile_enable(on=True, hops_only=False):
    """Time every stage and hop launch with HIP events on its stream (with
    hops_only, the hop launches alone)."""
    _check(load().ahr_profile_enable((2 if hops_only else 1) if on else 0))


def profile_read(reset: bool = True) -> dict:
    p = _Profile()
    _check(load().ahr_profile_read(ctypes.byref(p), 1 if reset else 0))
    return {n: getattr(p, n) for n, _ in _Profile._fields_}


def mlp_forward(params, feats, out=None, stream=None):
    """o = MLP(feats) for feature rows feats [n, 8] (matrix-core evaluation)."""
    n = feats.shape[0]
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=feats.device)
    _check(load().ahr_mlp_forward(_ptr(params), _ptr(feats), n, _ptr(out), _stream(stream)))
    return out


def mlp_loss_grad(params, feats, target, grad=None, loss=None, rounding=True, stream=None):
    """(grad, loss) of mean (MLP(feats) - target)^2; both stay on the device.
    rounding=False: float32 operands instead of the bfloat16 rounding points."""
    n = feats.shape[0]
    if grad is None:
        grad = torch.empty(MLP_NPARAM, dtype=torch.float32, device=params.device)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float64, device=params.device)
    _check(load().ahr_mlp_loss_grad(_ptr(params), _ptr(feats), _ptr(target), n, _ptr(grad), _ptr(loss),
                                    1 if rounding else 0, _stream(stream)))
    return grad, loss


def mlp_adam(params, m, v, grad, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(load().ahr_mlp_adam(_ptr(params), _ptr(m), _ptr(v), _ptr(grad), step, lr, beta1, beta2, eps,
                               _stream(stream)))


class Mlp:
    """A learned-filter model: float32 parameters on the device, the linear
    weights beta of the input and the three hops (h0..h3), and whether it met
    its validation bound."""

    def __init__(self, params, beta=(0.0, 0.0, 0.0, 1.0), validated=True):
        self.params = params
        self.beta = tuple(float(b) for b in beta)
        if len(self.beta) != 4:
            raise ValueError("beta holds the weights of h0, h1, h2, h3")
        self.validated = bool(validated)

    def c(self):
        return _Mlp(self.params.data_ptr(), (ctypes.c_float * 4)(*self.beta), 1 if self.validated else 0)

    @classmethod
    def load(cls, path, device="cuda"):
        """A model written by the trainer (JSON; nothing in it is executed)."""
        import json
        with open(path) as f:
            doc = json.load(f)
        if doc.get("format") != "ahr-mlp-2" or int(doc["nparam"]) != MLP_NPARAM:
            raise ValueError(f"{path}: not a model of this network shape")
        p = torch.tensor(np.asarray(doc["params"], np.float32)).to(device)
        m = cls(p, doc["beta"], doc["validated"])
        m.summary = doc.get("summary", {})
        return m


class Netlist:
    """A netlist resident on the device (the arrays the C ABI points to)."""

    def __init__(self, arrays: dict, device="cuda"):
        dev = torch.device(device)
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to(dev, dt)
        self.n_inst = int(arrays["n_inst"])
        self.net_ptr = t(arrays["net_ptr"], torch.int32)
        self.pin_node = t(arrays["pin_node"], torch.int32)
        self.pin_off = t(arrays["pin_off"], torch.float32)
        self.node_flags = t(arrays["node_flags"], torch.uint8)
        self.node_size = t(arrays["node_size"], torch.float32)
        nw = arrays.get("net_w")
        self.net_w = None if nw is None else t(nw, torch.float32)
        self.die = [float(v) for v in np.asarray(arrays["die"], np.float32)]
        self.c = _Netlist(self.n_inst, self.net_ptr.numel() - 1, self.pin_node.numel(), 0,
                          self.net_ptr.data_ptr(), self.pin_node.data_ptr() if self.pin_node.numel() else 0,
                          self.pin_off.data_ptr(), self.net_w.data_ptr() if self.net_w is not None else 0,
                          self.node_flags.data_ptr(), self.node_size.data_ptr(), (ctypes.c_float * 4)(*self.die))


def hpwl(netlist: Netlist, g, out=None, stream=None):
    """Per column pair HPWL of the placements in g [n_inst, C] (device float64 [C/2])."""
    if out is None:
        out = torch.empty(g.shape[1] // 2, dtype=torch.float64, device=g.device)
    _check(load().ahr_hpwl(ctypes.byref(netlist.c), _ptr(g), g.shape[1], _ptr(out), _stream(stream)))
    return out


def hpwl_noalloc(netlist: Netlist, g, out, stream=None):
    """ahr_hpwl with the library's fixed partial-sum buffer: no allocation
    (the caller passes `out`, device float64 [C/2]); calls that overlap on one
    device race."""
    _check(load().ahr_hpwl_noalloc(ctypes.byref(netlist.c), _ptr(g), g.shape[1], _ptr(out), _stream(stream)))
    return out


def hint_params(nbx=8, nby=8, detection_ratio=0.1, bin_capacity=1.0, mu=4.0, clique_max=10, flags=ALL_HINTS,
                prune_tau=0.0):
    return _HintParams(nbx, nby, detection_ratio, bin_capacity, mu, clique_max, flags, prune_tau)


def filter_spec(ks=(4,), alphas=(1.0,), sigma=0.0, lambda_mode=LAMBDA_GERSHGORIN, lambda_fixed=2.0):
    ks, alphas = list(ks), list(alphas)
    assert len(ks) == len(alphas) and 1 <= len(ks) <= 4
    k = (ctypes.c_int32 * 4)(*(ks + [0] * (4 - len(ks))))
    a = (ctypes.c_float * 4)(*(alphas + [0.0] * (4 - len(alphas))))
    return _FilterSpec(len(ks), k, a, sigma, lambda_mode, lambda_fixed)


def gift_spec(ks=(2, 2, 4), sigmas=(2.0, 4.0, 4.0), alphas=(0.2, 0.3, 0.5)):
    """GiFt bank: bands (k, sigma) with weights alpha (Section IV)."""
    ks, sigmas, alphas = list(ks), list(sigmas), list(alphas)
    assert len(ks) == len(sigmas) == len(alphas) and 1 <= len(ks) <= 4
    pad = 4 - len(ks)
    return _GiftSpec(len(ks), (ctypes.c_int32 * 4)(*(ks + [0] * pad)), (ctypes.c_float * 4)(*(alphas + [0.0] * pad)),
                     (ctypes.c_float * 4)(*(sigmas + [0.0] * pad)))


def workspace_size(netlist: Netlist, params, ncols, stream=None) -> int:
    """Bytes of device workspace a graph of this netlist needs (ahr_graph_workspace_size)."""
    n = ctypes.c_size_t()
    _check(load().ahr_graph_workspace_size(ctypes.byref(netlist.c), ctypes.byref(params), ncols, _stream(stream),
                                           ctypes.byref(n)))
    return n.value


def refine(netlist: Netlist, params, spec, g0, T_hint, gamma, out=None, ws=None, stream=None):
    """Algorithm 1 end to end (graph built, refined and freed in one call);
    ws: an optional device workspace (uint8 tensor) for all its memory."""
    if out is None:
        out = torch.empty_like(g0)
    _check(load().ahr_refine(ctypes.byref(netlist.c), ctypes.byref(params), ctypes.byref(spec), _ptr(g0), g0.shape[1],
                             T_hint, gamma, _ptr(out), _ptr(ws), 0 if ws is None else ws.numel(), _stream(stream)))
    return out


class Graph:
    """Owner of an ahr_graph handle (ahr_graph_build ... ahr_graph_destroy).
    ws: an optional device workspace (uint8 tensor, kept alive by the
    handle) that all of the graph's device memory is carved from."""

    def __init__(self, netlist: Netlist, params, g=None, stream=None, ws=None):
        lib = load()
        self.netlist = netlist
        self.params = params
        self.ws = ws
        h = ctypes.c_void_p()
        ncols = 0 if g is None else g.shape[1]
        _check(lib.ahr_graph_build(ctypes.byref(netlist.c), ctypes.byref(params), _ptr(g), ncols, _ptr(ws),
                                   0 if ws is None else ws.numel(), _stream(stream), ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            load().ahr_graph_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def update_hints(self, g, stream=None):
        _check(load().ahr_graph_update_hints(self.h, _ptr(g), g.shape[1], _stream(stream)))

    def info(self) -> dict:
        i = _GraphInfo()
        _check(load().ahr_graph_get_info(self.h, ctypes.byref(i)))
        return {n: getattr(i, n) for n, _ in _GraphInfo._fields_}

    def export(self, stream=None) -> dict:
        inf = self.info()
        n, nn, nh = inf["n_tot"], inf["nnz_net"], inf["nnz_hint"]
        out = dict(net_row_ptr=np.zeros(n + 1, np.int32), net_col=np.zeros(max(nn, 1), np.int32),
                   net_q=np.zeros(max(nn, 1), np.int64), hint_row_ptr=np.zeros(n + 1, np.int32),
                   hint_col=np.zeros(max(nh, 1), np.int32), hint_val=np.zeros(max(nh, 1), np.float32),
                   degree=np.zeros(n, np.float64), scale=np.zeros(n, np.float32),
                   lambda_up=np.zeros(1, np.float32))
        h = _GraphHost(*[a.ctypes.data for a in out.values()])
        _check(load().ahr_graph_export(self.h, ctypes.byref(h), _stream(stream)))
        out["net_col"] = out["net_col"][:nn]
        out["net_q"] = out["net_q"][:nn]
        out["hint_col"] = out["hint_col"][:nh]
        out["hint_val"] = out["hint_val"][:nh]
        out["lambda_up"] = float(out["lambda_up"][0])
        return out

    def filter(self, spec, x, out=None, stream=None):
        if out is None:
            out = torch.empty_like(x)
        _check(load().ahr_filter(self.h, ctypes.byref(spec), _ptr(x), _ptr(out), x.shape[1], _stream(stream)))
        return out

    def gift(self, spec, x, out=None, stream=None):
        """GiFt's bank on the netlist graph (no area hints), fixed rows reset."""
        if out is None:
            out = torch.empty_like(x)
        _check(load().ahr_gift(self.h, ctypes.byref(spec), _ptr(x), _ptr(out), x.shape[1], _stream(stream)))
        return out

    def refine(self, spec, g0, T_hint, gamma, out=None, stream=None):
        if out is None:
            out = torch.empty_like(g0)
        _check(load().ahr_graph_refine(self.h, ctypes.byref(spec), _ptr(g0), g0.shape[1], T_hint, gamma, _ptr(out),
                                       _stream(stream)))
        return out

    def refine_learned(self, spec, model, g0, T_hint, gamma, out=None, stream=None):
        """(out, used_fallback) of Algorithm 1 with the learned filter."""
        if out is None:
            out = torch.empty_like(g0)
        fb = ctypes.c_int32(-1)
        mc = model.c()
        _check(load().ahr_refine_learned(self.h, ctypes.byref(spec), ctypes.byref(mc), _ptr(g0), g0.shape[1], T_hint,
                                         gamma, _ptr(out), ctypes.byref(fb), _stream(stream)))
        return out, bool(fb.value)

    def filter_learned(self, spec, model, x, out=None, stream=None):
        """(out, used_fallback) of the learned filter."""
        if out is None:
            out = torch.empty_like(x)
        fb = ctypes.c_int32(-1)
        mc = model.c()
        _check(load().ahr_filter_learned(self.h, ctypes.byref(spec), ctypes.byref(mc), _ptr(x), _ptr(out),
                                         x.shape[1], ctypes.byref(fb), _stream(stream)))
        return out, bool(fb.value)

    def features(self, spec, x, stream=None):
        """(feats [n*C, 8], hops [4, n, C] (h0..h3), stats [3, C] (m, s, r)) of the
        surrogate for signal x."""
        n, C = x.shape
        feats = torch.empty((n * C, MLP_FEATURE_STRIDE), dtype=torch.float32, device=x.device)
        hops = torch.empty((4, n, C), dtype=torch.float32, device=x.device)
        stats = torch.empty((3, C), dtype=torch.float32, device=x.device)
        _check(load().ahr_filter_features(self.h, ctypes.byref(spec), _ptr(x), C, _ptr(feats), _ptr(hops),
                                          _ptr(stats), _stream(stream)))
        return feats, hops, stats

    def hpwl(self, g, out=None, stream=None):
        """HPWL of the graph's netlist (ahr_hpwl needs only the netlist)."""
        return hpwl(self.netlist, g, out, stream)


class Wirelength:
    """Owner of an ahr_wl handle: the WA wirelength and its gradient
    (ahr_wl_create ... ahr_wl_destroy)."""

    def __init__(self, netlist: Netlist, stream=None):
        self.netlist = netlist
        h = ctypes.c_void_p()
        _check(load().ahr_wl_create(ctypes.byref(netlist.c), _stream(stream), ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            load().ahr_wl_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def wa(self, g, gamma, grad=True, stream=None):
        """(wl [C/2] float64, grad [n_inst, C] float32 or None) on the device."""
        wl = torch.empty(g.shape[1] // 2, dtype=torch.float64, device=g.device)
        gr = torch.empty_like(g) if grad else None
        _check(load().ahr_wa(self.h, _ptr(g), g.shape[1], float(gamma), _ptr(wl), _ptr(gr), _stream(stream)))
        return wl, gr


class Batch:
    """Owner of an ahr_batch handle: many netlists filtered as one
    block-diagonal operator (ahr_batch_build ... ahr_batch_destroy).

    `pos` is the members' placements concatenated in member order
    ([sum n_inst, C] on the device); filter inputs and outputs use the same
    layout.  `params` is one hint-parameter struct or one per member."""

    def __init__(self, netlists, params, pos, stream=None):
        lib = load()
        self.netlists = list(netlists)
        n = len(self.netlists)
        if not isinstance(params, (list, tuple)):
            params = [params] * n
        self._nls = (_Netlist * n)(*[nl.c for nl in self.netlists])
        self._hps = (_HintParams * n)(*params)
        self.offsets = np.concatenate([[0], np.cumsum([nl.n_inst for nl in self.netlists])]).astype(np.int64)
        h = ctypes.c_void_p()
        _check(lib.ahr_batch_build(ctypes.cast(self._nls, ctypes.c_void_p), ctypes.cast(self._hps, ctypes.c_void_p),
                                   n, _ptr(pos), pos.shape[1], _stream(stream), ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            load().ahr_batch_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        i = _BatchInfo()
        _check(load().ahr_batch_get_info(self.h, ctypes.byref(i)))
        return {n: getattr(i, n) for n, _ in _BatchInfo._fields_}

    def filter(self, spec, x, out=None, use_graph=True, stream=None):
        if out is None:
            out = torch.empty_like(x)
        _check(load().ahr_batch_filter(self.h, ctypes.byref(spec), _ptr(x), _ptr(out), x.shape[1],
                                       1 if use_graph else 0, _stream(stream)))
        return out

    def set_config(self, ncols, lanes_per_row=0, col_tile=0):
        _check(load().ahr_batch_set_config(self.h, ncols, lanes_per_row, col_tile))

    def get_config(self, ncols):
        lanes, ct = ctypes.c_int32(), ctypes.c_int32()
        _check(load().ahr_batch_get_config(self.h, ncols, ctypes.byref(lanes), ctypes.byref(ct)))
        return lanes.value, ct.value

    def autotune(self, spec, ncols, stream=None):
        """(lanes_per_row, col_tile, ms) of the fastest launch shape, now the batch's configuration."""
        lanes, ct, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_float()
        _check(load().ahr_batch_autotune(self.h, ctypes.byref(spec), ncols, _stream(stream), ctypes.byref(lanes),
                                         ctypes.byref(ct), ctypes.byref(ms)))
        return lanes.value, ct.value, ms.value
