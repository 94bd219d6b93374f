"""Python binding of libtucker (MI355X dense Tucker / HOOI, arXiv 1707.05594).

Thin ctypes marshalling over the C ABI declared in include/tucker.h: every
computation happens in the HIP library.  PyTorch is used only to hold device
memory and to name the stream; tensors are passed by data pointer.

The names follow the C ABI: ``ttm_tree_plan``, ``hooi_init``,
``hooi_iterate``, ``tucker_error`` plus the inspection and kernel-level calls.
If the library is missing this module raises at first use -- there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtucker.so")

TK_OK, TK_EINVAL, TK_ENOMEM, TK_EDEVICE, TK_ENUMERIC, TK_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
TK_F64, TK_F32, TK_BF16, TK_F16 = 0, 1, 2, 3
TK_C_FP64, TK_C_FP32, TK_C_BF16, TK_C_BF16X3 = 0, 1, 2, 3
TREE_KINDS = {"dp": 0, "chain": 1, "chain_k": 2, "chain_h": 3, "balanced": 4}
TK_TILE_AUTO, TK_TILE_STAGED, TK_TILE_SPLITK, TK_TILE_COUNT = 0, 1, 2, 3
TK_TILE_PAIR = 3
TK_FEATURES = 13
COMPUTE = {"fp64": TK_C_FP64, "fp32": TK_C_FP32, "bf16": TK_C_BF16, "bf16x3": TK_C_BF16X3}
DTYPES = {"f64": TK_F64, "f32": TK_F32, "bf16": TK_BF16, "f16": TK_F16}
MAX_MODES = 12


class TuckerError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libtucker error {code}: {msg}")
        self.code = code


class TkNode(ctypes.Structure):
    _fields_ = [("parent", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("is_leaf", ctypes.c_int32), ("depth", ctypes.c_int32),
                ("in_card", ctypes.c_uint64), ("out_card", ctypes.c_uint64),
                ("macs", ctypes.c_uint64), ("pre_mask", ctypes.c_uint32),
                ("pad_", ctypes.c_uint32)]


class TkNodeView(ctypes.Structure):
    _fields_ = [("node", ctypes.c_int32), ("in_dtype", ctypes.c_int32),
                ("out_dtype", ctypes.c_int32), ("compute", ctypes.c_int32),
                ("A", ctypes.c_int64), ("L", ctypes.c_int64), ("B", ctypes.c_int64),
                ("K", ctypes.c_int64)]


_lib = None
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i64p = ctypes.POINTER(ctypes.c_int64)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_fp = ctypes.POINTER(ctypes.c_float)

_SIGS = {
    "ttm_tree_plan": ([ctypes.c_int, _i64p, _i64p, ctypes.c_int, ctypes.c_int,
                       ctypes.POINTER(_vp)], ctypes.c_int),
    "tk_plan_count": ([_vp, _ip], ctypes.c_int),
    "tk_plan_cost": ([_vp, ctypes.c_int, _u64p], ctypes.c_int),
    "tk_plan_string": ([_vp, ctypes.c_int, ctypes.c_char_p, ctypes.c_size_t], ctypes.c_int),
    "tk_plan_nodes": ([_vp, ctypes.c_int, ctypes.POINTER(TkNode), ctypes.c_int, _ip],
                      ctypes.c_int),
    "tk_plan_stats": ([_vp, _u64p, _u64p], ctypes.c_int),
    "tk_plan_workspace": ([_vp, ctypes.c_int, _u64p], ctypes.c_int),
    "tk_plan_select": ([_vp, ctypes.c_int], ctypes.c_int),
    "tk_plan_free": ([_vp], None),
    "hooi_init": ([ctypes.c_int, _i64p, _i64p, ctypes.c_int, _vp, _vp, ctypes.c_int, _dp, _vp,
                   ctypes.POINTER(_vp)], ctypes.c_int),
    "hooi_init_sthosvd": ([ctypes.c_int, _i64p, _i64p, ctypes.c_int, _vp, _vp, ctypes.c_int,
                           ctypes.POINTER(ctypes.c_int), _vp, ctypes.POINTER(_vp)],
                          ctypes.c_int),
    "hooi_iterate": ([_vp, ctypes.c_int, _dp], ctypes.c_int),
    "tucker_error": ([_vp, _dp, _dp, _dp], ctypes.c_int),
    "tucker_error_explicit": ([_vp, _dp], ctypes.c_int),
    "tk_get_factor": ([_vp, ctypes.c_int, _dp], ctypes.c_int),
    "tk_get_core": ([_vp, _dp], ctypes.c_int),
    "tk_set_factors": ([_vp, _dp], ctypes.c_int),
    "tk_tree_pass": ([_vp], ctypes.c_int),
    "tk_get_leaf": ([_vp, ctypes.c_int, _dp], ctypes.c_int),
    "tk_get_gram": ([_vp, ctypes.c_int, _dp], ctypes.c_int),
    "tk_profile_tree": ([_vp, ctypes.POINTER(ctypes.c_float), ctypes.c_int, _ip], ctypes.c_int),
    "tk_eig_iterations": ([_vp, _ip], ctypes.c_int),
    "hooi_free": ([_vp], None),
    "tk_ttm": ([ctypes.c_int, ctypes.c_int, _vp, _i64, _i64, _i64, _vp, _i64, _vp, _vp],
               ctypes.c_int),
    "tk_gram": ([ctypes.c_int, _vp, _i64, _i64, _i64, _vp, _vp], ctypes.c_int),
    "tk_grid_count": ([_i64, ctypes.c_int, ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
    "tk_plan_grids": ([_vp, ctypes.c_int, _i64, ctypes.c_int, _ip, _ip, ctypes.c_int,
                       ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
    "tk_ttm_pair": ([ctypes.c_int, ctypes.c_int, _vp, _i64, _i64, _i64, _i64, _i64, _vp, _i64,
                     _vp, _i64, _vp, _vp, _vp], ctypes.c_int),
    "tk_gram_noalloc": ([ctypes.c_int, _vp, _i64, _i64, _i64, _vp, _vp], ctypes.c_int),
    "tk_eig_leading": ([ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, _vp, _vp],
                       ctypes.c_int),
    "tk_eig_full": ([ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, _vp],
                    ctypes.c_int),
    "tk_ttm_features": ([_i64, _i64, _i64, _i64, ctypes.c_int, ctypes.c_int, ctypes.c_int, _fp],
                        ctypes.c_int),
    "tk_pair_features": ([_i64, _i64, _i64, _i64, _i64, _i64, _i64, ctypes.c_int, ctypes.c_int,
                          _fp], ctypes.c_int),
    "tk_time_ttm_pair": ([ctypes.c_int, ctypes.c_int, _vp, _i64, _i64, _i64, _i64, _i64, _vp,
                          _i64, _vp, _i64, _vp, _vp, ctypes.c_int, _vp, _fp], ctypes.c_int),
    "tk_time_ttm": ([ctypes.c_int, ctypes.c_int, _vp, _i64, _i64, _i64, _vp, _i64, _vp,
                     ctypes.c_int, ctypes.c_int, _vp, _fp], ctypes.c_int),
    "tk_plan_set_tiles": ([_vp, ctypes.c_int, _ip, ctypes.c_int], ctypes.c_int),
    "tk_plan_get_tiles": ([_vp, ctypes.c_int, _ip, ctypes.c_int, _ip], ctypes.c_int),
    "tk_mlp_param_count": ([ctypes.c_int, ctypes.c_int], ctypes.c_int64),
    "tk_mlp_create": ([ctypes.c_int, ctypes.c_int, _fp, ctypes.POINTER(_vp)], ctypes.c_int),
    "tk_mlp_set_norm": ([_vp, _fp, _fp], ctypes.c_int),
    "tk_mlp_fit_norm": ([_vp, _fp, ctypes.c_int], ctypes.c_int),
    "tk_mlp_get_params": ([_vp, _fp], ctypes.c_int),
    "tk_mlp_set_params": ([_vp, _fp], ctypes.c_int),
    "tk_mlp_forward": ([_vp, _fp, ctypes.c_int, _fp], ctypes.c_int),
    "tk_mlp_loss_grad": ([_vp, _fp, _fp, ctypes.c_int, _fp, _fp], ctypes.c_int),
    "tk_mlp_train": ([_vp, _fp, _fp, ctypes.c_int, ctypes.c_int, ctypes.c_float, _fp],
                     ctypes.c_int),
    "tk_mlp_free": ([_vp], None),
    "tk_plan_learned": ([_vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_double, _ip, _dp],
                        ctypes.c_int),
    "tk_plan_node_views": ([_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_int,
                            _ip], ctypes.c_int),
    "tk_plan_root_pair": ([_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _i64p, _ip],
                          ctypes.c_int),
    "hooi_batch_init": ([ctypes.c_int, _ip, _i64p, _i64p, ctypes.c_int, ctypes.POINTER(_vp),
                         ctypes.c_int, _vp, ctypes.POINTER(_vp)], ctypes.c_int),
    "hooi_batch_iterate": ([_vp, ctypes.c_int, _dp], ctypes.c_int),
    "hooi_batch_error": ([_vp, _dp], ctypes.c_int),
    "hooi_batch_get_factor": ([_vp, ctypes.c_int, ctypes.c_int, _dp], ctypes.c_int),
    "hooi_batch_get_factors": ([_vp, _dp], ctypes.c_int),
    "hooi_batch_set_factors": ([_vp, _dp], ctypes.c_int),
    "hooi_batch_use_graph": ([_vp, ctypes.c_int], ctypes.c_int),
    "hooi_batch_tune": ([_vp, _ip, _fp], ctypes.c_int),
    "hooi_batch_stats": ([_vp, _u64p, _u64p, _ip, _ip], ctypes.c_int),
    "hooi_batch_free": ([_vp], None),
    "tk_last_error": ([], ctypes.c_char_p),
}


def lib():
    """Load libtucker.so (built by paper_1707_05594_amd.build); raise if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1707_05594_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def _check(rc):
    if rc != TK_OK:
        raise TuckerError(rc, lib().tk_last_error().decode(errors="replace"))


def _arr64(vals):
    return (ctypes.c_int64 * len(vals))(*[int(v) for v in vals])


# ----------------------------------------------------------------------------- planning --
class Plan:
    """A TTM-tree plan (host only).  Rank 0 is the selected tree unless select() is used."""

    def __init__(self, handle, L, K):
        self._h = handle
        self.L = tuple(int(x) for x in L)
        self.K = tuple(int(x) for x in K)

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.tk_plan_free(self._h)
            self._h = None

    @property
    def handle(self):
        return self._h

    @property
    def count(self):
        n = ctypes.c_int()
        _check(lib().tk_plan_count(self._h, ctypes.byref(n)))
        return n.value

    def cost(self, rank=0):
        c = ctypes.c_uint64()
        _check(lib().tk_plan_cost(self._h, rank, ctypes.byref(c)))
        return int(c.value)

    def string(self, rank=0):
        buf = ctypes.create_string_buffer(1 << 16)
        _check(lib().tk_plan_string(self._h, rank, buf, len(buf)))
        return buf.value.decode()

    def nodes(self, rank=0):
        n = ctypes.c_int()
        _check(lib().tk_plan_nodes(self._h, rank, None, 0, ctypes.byref(n)))
        arr = (TkNode * n.value)()
        _check(lib().tk_plan_nodes(self._h, rank, arr, n.value, ctypes.byref(n)))
        return [dict(parent=x.parent, mode=x.mode, is_leaf=bool(x.is_leaf), depth=x.depth,
                     in_card=int(x.in_card), out_card=int(x.out_card), macs=int(x.macs),
                     pre_mask=int(x.pre_mask)) for x in arr]

    def stats(self):
        e, l = ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().tk_plan_stats(self._h, ctypes.byref(e), ctypes.byref(l)))
        return int(e.value), int(l.value)

    def workspace(self, rank=0):
        w = ctypes.c_uint64()
        _check(lib().tk_plan_workspace(self._h, rank, ctypes.byref(w)))
        return int(w.value)

    def select(self, rank):
        _check(lib().tk_plan_select(self._h, rank))

    def set_tiles(self, rank, tiles):
        arr = (ctypes.c_int * len(tiles))(*[int(t) for t in tiles])
        _check(lib().tk_plan_set_tiles(self._h, rank, arr, len(tiles)))

    def tiles(self, rank=0):
        n = ctypes.c_int()
        _check(lib().tk_plan_get_tiles(self._h, rank, None, 0, ctypes.byref(n)))
        arr = (ctypes.c_int * n.value)()
        _check(lib().tk_plan_get_tiles(self._h, rank, arr, n.value, ctypes.byref(n)))
        return list(arr)

    def grids(self, P, kind="dynamic", rank=0):
        """Processor grids for P processors (Sec. 4): (volume, root grid,
        per-node grids in nodes() order); kind "static" or "dynamic"."""
        N = len(self.L)
        n = len(self.nodes(rank))
        root = (ctypes.c_int * N)()
        per = (ctypes.c_int * (n * N))()
        vol = ctypes.c_uint64()
        _check(lib().tk_plan_grids(self._h, int(rank), int(P),
                                   {"static": 0, "dynamic": 1}[kind], root, per, n,
                                   ctypes.byref(vol)))
        return (int(vol.value), tuple(root),
                [tuple(per[u * N:(u + 1) * N]) for u in range(n)])

    def node_views(self, rank=0, tdtype="f32", compute="fp32"):
        """The internal nodes' TTM views as the engine runs them: dicts of
        node, A, L, B, K, in_dtype, out_dtype, compute (names)."""
        n = ctypes.c_int()
        _check(lib().tk_plan_node_views(self._h, rank, DTYPES[tdtype], COMPUTE[compute], None,
                                        0, ctypes.byref(n)))
        arr = (TkNodeView * n.value)()
        _check(lib().tk_plan_node_views(self._h, rank, DTYPES[tdtype], COMPUTE[compute], arr,
                                        n.value, ctypes.byref(n)))
        dn = {v: k for k, v in DTYPES.items()}
        cn = {v: k for k, v in COMPUTE.items()}
        return [dict(node=x.node, A=int(x.A), L=int(x.L), B=int(x.B), K=int(x.K),
                     in_dtype=dn[x.in_dtype], out_dtype=dn[x.out_dtype],
                     compute=cn[x.compute]) for x in arr]

    def root_pair(self, rank=0, tdtype="f32", compute="fp32"):
        """(A, Lp, M, Lq, B, Kp, Kq) of the two root children, and whether a
        pair kernel takes them; (None, False) unless the root has exactly two
        internal children."""
        v = (ctypes.c_int64 * 7)()
        f = ctypes.c_int()
        _check(lib().tk_plan_root_pair(self._h, rank, DTYPES[tdtype], COMPUTE[compute], v,
                                       ctypes.byref(f)))
        if v[0] == 0:
            return None, False
        return tuple(int(x) for x in v), bool(f.value)

    def learned(self, model, tdtype="f32", compute="fp32", margin=0.02):
        """Select a held tree and per-node kernels by the cost model; returns
        (chosen rank, predicted ms per rank)."""
        import numpy as np
        chosen = ctypes.c_int()
        pred = np.zeros(self.count, dtype=np.float64)
        _check(lib().tk_plan_learned(self._h, model.handle, DTYPES[tdtype], COMPUTE[compute],
                                     float(margin), ctypes.byref(chosen),
                                     pred.ctypes.data_as(_dp)))
        return chosen.value, pred


def grid_count(P, N):
    """psi(P, N): the number of N-dimensional grids of P processors (Sec. 4.2)."""
    c = ctypes.c_uint64()
    _check(lib().tk_grid_count(int(P), int(N), ctypes.byref(c)))
    return int(c.value)


def ttm_tree_plan(L, K, kind="dp", topk=1) -> Plan:
    """Plan a TTM-tree for lengths L and core lengths K (kind: dp, chain, chain_k,
    chain_h, balanced)."""
    h = _vp()
    _check(lib().ttm_tree_plan(len(L), _arr64(L), _arr64(K), TREE_KINDS[kind], int(topk),
                               ctypes.byref(h)))
    return Plan(h, L, K)


# ----------------------------------------------------------------------------- device side --
def _torch():
    import torch
    return torch


def _dtype_code(t):
    torch = _torch()
    m = {torch.float64: TK_F64, torch.float32: TK_F32, torch.bfloat16: TK_BF16,
         torch.float16: TK_F16}
    if t.dtype not in m:
        raise TypeError(f"unsupported dtype {t.dtype}")
    return m[t.dtype]


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return _vp(s.cuda_stream)


def _dev_ptr(t):
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return _vp(t.data_ptr())


class Context:
    """HOOI context on a device tensor T (borrowed: keep T alive)."""

    def __init__(self, T, K, plan=None, compute="fp32", F0=None, stream=None, init="hosvd",
                 order=None):
        import numpy as np
        self.T = T
        self.L = tuple(int(x) for x in T.shape)
        self.K = tuple(int(x) for x in K)
        self.N = len(self.L)
        self._stream = stream
        f0p = None
        if F0 is not None:
            flat = np.concatenate([np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
                                   for f in F0])
            self._f0 = flat
            f0p = flat.ctypes.data_as(_dp)
        h = _vp()
        comp = COMPUTE[compute] if isinstance(compute, str) else int(compute)
        if init == "sthosvd":
            if F0 is not None:
                raise ValueError("F0 and init='sthosvd' exclude each other")
            ordp = None
            if order is not None:
                ordp = (ctypes.c_int * self.N)(*[int(n) for n in order])
            _check(lib().hooi_init_sthosvd(self.N, _arr64(self.L), _arr64(self.K),
                                           _dtype_code(T), _dev_ptr(T),
                                           plan.handle if plan is not None else None, comp,
                                           ordp, _stream_ptr(stream), ctypes.byref(h)))
        elif init == "hosvd":
            _check(lib().hooi_init(self.N, _arr64(self.L), _arr64(self.K), _dtype_code(T),
                                   _dev_ptr(T), plan.handle if plan is not None else None,
                                   comp, f0p, _stream_ptr(stream), ctypes.byref(h)))
        else:
            raise ValueError(f"unknown init {init!r}")
        self._h = h

    def __del__(self):
        self.free()

    def free(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hooi_free(self._h)
            self._h = None

    def iterate(self, iters=1):
        errs = (ctypes.c_double * iters)()
        _check(lib().hooi_iterate(self._h, iters, errs))
        return list(errs)

    def error(self):
        e, nt, ng = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(lib().tucker_error(self._h, ctypes.byref(e), ctypes.byref(nt), ctypes.byref(ng)))
        return e.value, nt.value, ng.value

    def error_explicit(self):
        e = ctypes.c_double()
        _check(lib().tucker_error_explicit(self._h, ctypes.byref(e)))
        return e.value

    def factor(self, n):
        import numpy as np
        out = np.empty((self.L[n], self.K[n]), dtype=np.float64)
        _check(lib().tk_get_factor(self._h, n, out.ctypes.data_as(_dp)))
        return out

    def factors(self):
        return [self.factor(n) for n in range(self.N)]

    def core(self):
        import numpy as np
        out = np.empty(self.K, dtype=np.float64)
        _check(lib().tk_get_core(self._h, out.ctypes.data_as(_dp)))
        return out

    def set_factors(self, F):
        import numpy as np
        flat = np.concatenate([np.ascontiguousarray(f, dtype=np.float64).reshape(-1) for f in F])
        _check(lib().tk_set_factors(self._h, flat.ctypes.data_as(_dp)))

    def tree_pass(self):
        _check(lib().tk_tree_pass(self._h))

    def leaf(self, n):
        import numpy as np
        shape = tuple(self.L[j] if j == n else self.K[j] for j in range(self.N))
        out = np.empty(shape, dtype=np.float64)
        _check(lib().tk_get_leaf(self._h, n, out.ctypes.data_as(_dp)))
        return out

    def gram(self, n):
        import numpy as np
        out = np.empty((self.L[n], self.L[n]), dtype=np.float64)
        _check(lib().tk_get_gram(self._h, n, out.ctypes.data_as(_dp)))
        return out

    def eig_iterations(self):
        arr = (ctypes.c_int * self.N)()
        _check(lib().tk_eig_iterations(self._h, arr))
        return list(arr)

    def profile_tree(self):
        n = ctypes.c_int()
        _check(lib().tk_profile_tree(self._h, None, 0, ctypes.byref(n)))
        arr = (ctypes.c_float * n.value)()
        _check(lib().tk_profile_tree(self._h, arr, n.value, ctypes.byref(n)))
        return list(arr)


def hooi_init(T, K, plan=None, compute="fp32", F0=None, stream=None, init="hosvd",
              order=None) -> Context:
    """Create a HOOI context: HOSVD start (init="hosvd") unless F0 (list of
    L_n x K_n) is given, or STHOSVD (init="sthosvd", modes in `order`)."""
    return Context(T, K, plan=plan, compute=compute, F0=F0, stream=stream, init=init,
                   order=order)


def hooi_iterate(ctx: Context, iters=1):
    """Run `iters` HOOI invocations; returns the relative error after each."""
    return ctx.iterate(iters)


def tucker_error(ctx: Context):
    """(relative error, ||T||, ||G||) of the current decomposition."""
    return ctx.error()


# ----------------------------------------------------------------------------- kernel level --
def ttm(inp, A, L, B, F, K, out, compute="fp32", stream=None):
    """Out[a,k,b] = sum_l F[l,k] In[a,l,b] on device tensors."""
    _check(lib().tk_ttm(_dtype_code(inp), COMPUTE[compute], _dev_ptr(inp), int(A), int(L),
                        int(B), _dev_ptr(F), int(K), _dev_ptr(out), _stream_ptr(stream)))


def ttm_pair(inp, A, Lp, M, Lq, B, Fp, Kp, Fq, Kq, outp, outq, compute="fp32", stream=None):
    """Both root TTMs of `inp` viewed as [A, Lp, M, Lq, B] in one pass."""
    _check(lib().tk_ttm_pair(_dtype_code(inp), COMPUTE[compute], _dev_ptr(inp), int(A),
                             int(Lp), int(M), int(Lq), int(B), _dev_ptr(Fp), int(Kp),
                             _dev_ptr(Fq), int(Kq), _dev_ptr(outp), _dev_ptr(outq),
                             _stream_ptr(stream)))


def gram(Y, A, L, B, S, stream=None):
    """S (L x L FP64, device) = Gram of the mode unfolding of Y viewed as [A, L, B]."""
    _check(lib().tk_gram(_dtype_code(Y), _dev_ptr(Y), int(A), int(L), int(B), _dev_ptr(S),
                         _stream_ptr(stream)))


def gram_noalloc(Y, A, L, B, S, stream=None):
    """As gram(), with no device allocation (static scratch area; asynchronous)."""
    _check(lib().tk_gram_noalloc(_dtype_code(Y), _dev_ptr(Y), int(A), int(L), int(B),
                                 _dev_ptr(S), _stream_ptr(stream)))


def eig_leading(S, K, V0=None, F=None, evals=None, stream=None):
    """Leading K eigenpairs of count x L x L symmetric FP64 device matrices."""
    torch = _torch()
    if S.dim() == 2:
        S = S.unsqueeze(0)
    count, L, _ = S.shape
    if F is None:
        F = torch.empty((count, L, K), dtype=torch.float64, device=S.device)
    if evals is None:
        evals = torch.empty((count, K), dtype=torch.float64, device=S.device)
    _check(lib().tk_eig_leading(count, L, K, _dev_ptr(S),
                                _dev_ptr(V0) if V0 is not None else None, _dev_ptr(F),
                                _dev_ptr(evals), _stream_ptr(stream)))
    return F, evals


def eig_full(S, K, F=None, evals=None, stream=None):
    """Leading K eigenpairs by the gap-free solver (tridiagonalisation + QL)."""
    torch = _torch()
    if S.dim() == 2:
        S = S.unsqueeze(0)
    count, L, _ = S.shape
    if F is None:
        F = torch.empty((count, L, K), dtype=torch.float64, device=S.device)
    if evals is None:
        evals = torch.empty((count, K), dtype=torch.float64, device=S.device)
    _check(lib().tk_eig_full(count, L, K, _dev_ptr(S), _dev_ptr(F), _dev_ptr(evals),
                             _stream_ptr(stream)))
    return F, evals


# ----------------------------------------------------------------------------- cost model --
def _f32(a):
    import numpy as np
    return np.ascontiguousarray(a, dtype=np.float32)


def ttm_features(A, L, B, K, in_dtype="f32", compute="fp32", tile=TK_TILE_AUTO):
    """Cost-model features of one TTM node (TK_FEATURES floats)."""
    import numpy as np
    out = np.zeros(TK_FEATURES, dtype=np.float32)
    _check(lib().tk_ttm_features(int(A), int(L), int(B), int(K), DTYPES[in_dtype],
                                 COMPUTE[compute], int(tile), out.ctypes.data_as(_fp)))
    return out


def pair_features(A, Lp, M, Lq, B, Kp, Kq, in_dtype="f32", compute="fp32"):
    """Cost-model features of a fused root pair (TK_FEATURES floats)."""
    import numpy as np
    out = np.zeros(TK_FEATURES, dtype=np.float32)
    _check(lib().tk_pair_features(int(A), int(Lp), int(M), int(Lq), int(B), int(Kp), int(Kq),
                                  DTYPES[in_dtype], COMPUTE[compute],
                                  out.ctypes.data_as(_fp)))
    return out


def time_ttm_pair(inp, A, Lp, M, Lq, B, Fp, Kp, Fq, Kq, outp, outq, compute="fp32", reps=5,
                  stream=None):
    """Average ms of `reps` fused root-pair launches (library timer)."""
    ms = ctypes.c_float()
    _check(lib().tk_time_ttm_pair(_dtype_code(inp), COMPUTE[compute], _dev_ptr(inp), int(A),
                                  int(Lp), int(M), int(Lq), int(B), _dev_ptr(Fp), int(Kp),
                                  _dev_ptr(Fq), int(Kq), _dev_ptr(outp), _dev_ptr(outq),
                                  int(reps), _stream_ptr(stream), ctypes.byref(ms)))
    return float(ms.value)


def time_ttm(inp, A, L, B, F, K, out, compute="fp32", tile=TK_TILE_AUTO, reps=5, stream=None):
    """Average time (ms) of the TTM node kernel on device tensors (HIP events)."""
    ms = ctypes.c_float()
    _check(lib().tk_time_ttm(_dtype_code(inp), COMPUTE[compute], _dev_ptr(inp), int(A), int(L),
                             int(B), _dev_ptr(F), int(K), _dev_ptr(out), int(tile), int(reps),
                             _stream_ptr(stream), ctypes.byref(ms)))
    return float(ms.value)


def mlp_param_count(in_dim, hidden):
    return int(lib().tk_mlp_param_count(int(in_dim), int(hidden)))


class MLP:
    """The cost model's MLP on the device (forward, backward, Adam in libtucker)."""

    def __init__(self, in_dim, hidden, params):
        p = _f32(params).reshape(-1)
        if p.size != mlp_param_count(in_dim, hidden):
            raise ValueError("wrong number of parameters")
        self.in_dim, self.hidden = int(in_dim), int(hidden)
        h = _vp()
        _check(lib().tk_mlp_create(self.in_dim, self.hidden, p.ctypes.data_as(_fp),
                                   ctypes.byref(h)))
        self._h = h

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.tk_mlp_free(self._h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def set_norm(self, mu, sigma):
        mu, sigma = _f32(mu), _f32(sigma)
        _check(lib().tk_mlp_set_norm(self._h, mu.ctypes.data_as(_fp), sigma.ctypes.data_as(_fp)))

    def fit_norm(self, X):
        """Standardise features by the per-feature mean and deviation of X."""
        X = _f32(X)
        _check(lib().tk_mlp_fit_norm(self._h, X.ctypes.data_as(_fp), X.shape[0]))

    def params(self):
        import numpy as np
        out = np.zeros(mlp_param_count(self.in_dim, self.hidden), dtype=np.float32)
        _check(lib().tk_mlp_get_params(self._h, out.ctypes.data_as(_fp)))
        return out

    def set_params(self, params):
        p = _f32(params).reshape(-1)
        _check(lib().tk_mlp_set_params(self._h, p.ctypes.data_as(_fp)))

    def forward(self, X):
        import numpy as np
        X = _f32(X)
        out = np.zeros(X.shape[0], dtype=np.float32)
        _check(lib().tk_mlp_forward(self._h, X.ctypes.data_as(_fp), X.shape[0],
                                    out.ctypes.data_as(_fp)))
        return out

    def loss_grad(self, X, y):
        import numpy as np
        X, y = _f32(X), _f32(y)
        loss = ctypes.c_float()
        g = np.zeros(mlp_param_count(self.in_dim, self.hidden), dtype=np.float32)
        _check(lib().tk_mlp_loss_grad(self._h, X.ctypes.data_as(_fp), y.ctypes.data_as(_fp),
                                      X.shape[0], ctypes.byref(loss), g.ctypes.data_as(_fp)))
        return float(loss.value), g

    def train(self, X, y, steps, lr):
        import numpy as np
        X, y = _f32(X), _f32(y)
        losses = np.zeros(int(steps), dtype=np.float32)
        _check(lib().tk_mlp_train(self._h, X.ctypes.data_as(_fp), y.ctypes.data_as(_fp),
                                  X.shape[0], int(steps), float(lr), losses.ctypes.data_as(_fp)))
        return losses


# ----------------------------------------------------------------------------- batched HOOI --
class Batch:
    """Batched HOOI over a list of device tensors (borrowed: keep them alive)."""

    def __init__(self, tensors, ranks, stream=None):
        import numpy as np
        self.tensors = list(tensors)
        self.L = [tuple(int(x) for x in t.shape) for t in self.tensors]
        self.K = [tuple(int(x) for x in k) for k in ranks]
        if len(self.K) != len(self.L):
            raise ValueError("one rank tuple per tensor")
        dts = {_dtype_code(t) for t in self.tensors}
        if len(dts) != 1:
            raise ValueError("all tensors must share one dtype")
        Ns = (ctypes.c_int * len(self.L))(*[len(l) for l in self.L])
        Ls = _arr64([x for l in self.L for x in l])
        Ks = _arr64([x for k in self.K for x in k])
        ptrs = (_vp * len(self.tensors))(*[_dev_ptr(t).value for t in self.tensors])
        h = _vp()
        _check(lib().hooi_batch_init(len(self.L), Ns, Ls, Ks, dts.pop(), ptrs, TK_C_FP32,
                                     _stream_ptr(stream), ctypes.byref(h)))
        self._h = h
        self.count = len(self.L)
        self._nf = sum(l * k for L_, K_ in zip(self.L, self.K) for l, k in zip(L_, K_))

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hooi_batch_free(self._h)
            self._h = None

    def iterate(self, iters=1):
        """errors[t][i]: error of tensor i's decomposition entering invocation t."""
        import numpy as np
        out = np.zeros((iters, self.count), dtype=np.float64)
        _check(lib().hooi_batch_iterate(self._h, int(iters), out.ctypes.data_as(_dp)))
        return out

    def error(self):
        import numpy as np
        out = np.zeros(self.count, dtype=np.float64)
        _check(lib().hooi_batch_error(self._h, out.ctypes.data_as(_dp)))
        return out

    def factor(self, i, n):
        import numpy as np
        out = np.empty((self.L[i][n], self.K[i][n]), dtype=np.float64)
        _check(lib().hooi_batch_get_factor(self._h, i, n, out.ctypes.data_as(_dp)))
        return out

    def factors(self):
        import numpy as np
        flat = np.empty(self._nf, dtype=np.float64)
        _check(lib().hooi_batch_get_factors(self._h, flat.ctypes.data_as(_dp)))
        return flat

    def set_factors(self, flat):
        import numpy as np
        flat = np.ascontiguousarray(flat, dtype=np.float64)
        _check(lib().hooi_batch_set_factors(self._h, flat.ctypes.data_as(_dp)))

    def use_graph(self, on=True):
        _check(lib().hooi_batch_use_graph(self._h, 1 if on else 0))

    def tune(self):
        import numpy as np
        bpc = ctypes.c_int()
        ms = np.zeros(5, dtype=np.float32)
        _check(lib().hooi_batch_tune(self._h, ctypes.byref(bpc), ms.ctypes.data_as(_fp)))
        return bpc.value, ms

    def stats(self):
        m, b = ctypes.c_uint64(), ctypes.c_uint64()
        lv, it = ctypes.c_int(), ctypes.c_int()
        _check(lib().hooi_batch_stats(self._h, ctypes.byref(m), ctypes.byref(b), ctypes.byref(lv),
                                      ctypes.byref(it)))
        return dict(tree_macs=int(m.value), tree_bytes=int(b.value), levels=lv.value,
                    ttm_items=it.value)

