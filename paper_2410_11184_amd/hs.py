"""Python binding of the C ABI in ``include/hs.h`` (argument marshalling only).

Every computation runs inside ``libhs.so`` (HIP kernels for gfx950 plus the
C++ host runtime).  If the library is missing the import fails loudly: there
is no CPU fallback.  PyTorch is used only to hand the library the current
HIP stream.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhs.so")

_u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_vp = ctypes.c_void_p

ERRORS = {
    -1: "HS_E_ARG", -2: "HS_E_PARAM", -3: "HS_E_LEVEL", -4: "HS_E_SCALE", -5: "HS_E_KEY",
    -6: "HS_E_OOM", -7: "HS_E_DEVICE", -8: "HS_E_RANGE", -9: "HS_E_STATE",
}


class HSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (ERRORS.get(code, code), msg))
        self.code = code
        self.name = ERRORS.get(code, str(code))


class hs_params(ctypes.Structure):
    _fields_ = [
        ("log_n", ctypes.c_int), ("n_q", ctypes.c_int), ("q_bits", ctypes.POINTER(ctypes.c_int)),
        ("n_p", ctypes.c_int), ("p_bits", ctypes.POINTER(ctypes.c_int)), ("digit", ctypes.c_int),
        ("hamming", ctypes.c_int), ("sigma", ctypes.c_double), ("log_scale", ctypes.c_int),
        ("user_top", ctypes.c_int), ("boot_cts_levels", ctypes.c_int), ("boot_evalmod_levels", ctypes.c_int),
        ("boot_stc_levels", ctypes.c_int), ("boot_K", ctypes.c_int), ("boot_double_angle", ctypes.c_int),
        ("boot_cos_degree", ctypes.c_int), ("boot_log_scale", ctypes.c_int),
    ]


class hs_ctx_info(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int) for n in
                ("log_n", "n", "slots", "n_q", "n_p", "top_level", "user_top", "dnum", "digit", "has_boot")]


class hs_softmax_opts(ctypes.Structure):
    _fields_ = [
        ("variant", ctypes.c_int), ("k", ctypes.c_int), ("exp_degree", ctypes.c_int),
        ("inv_degree_first", ctypes.c_int), ("inv_degree_mid", ctypes.c_int),
        ("inv_degree_last", ctypes.c_int), ("alpha", ctypes.c_double),
        ("power", ctypes.c_int), ("debug_stop", ctypes.c_int), ("newton_steps", ctypes.c_int),
        ("mask_mode", ctypes.c_int), ("approx", ctypes.c_int), ("merge", ctypes.c_int),
    ]


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libhs.so is not built: run python -c 'import __graft_entry__ as g; g.build()'")
    # torch first: its HIP runtime (same soname as the one libhs.so names) is
    # then the only one in the process, shared by the library and by the
    # device memory and streams that torch hands to it; loading the library
    # first would bring a second HIP runtime in beside torch's
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    S = ctypes.c_int
    L.hs_version.restype = ctypes.c_char_p
    L.hs_last_error.restype = ctypes.c_char_p
    sig = {
        "hs_ctx_create": [ctypes.POINTER(hs_params), S, _vp, ctypes.POINTER(_vp)],
        "hs_ctx_create_ex": [ctypes.POINTER(hs_params), S, _vp, _ALLOC_FN, _FREE_FN, _vp, ctypes.POINTER(_vp)],
        "hs_ctx_clone": [_vp, _vp, ctypes.POINTER(_vp)],
        "hs_ctx_get_info": [_vp, ctypes.POINTER(hs_ctx_info)],
        "hs_ctx_primes": [_vp, _u64p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)],
        "hs_sync": [_vp],
        "hs_keygen": [_vp, ctypes.c_uint64],
        "hs_add_rotation_keys": [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.c_size_t, S],
        "hs_key_export": [_vp, S, _u64p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)],
        "hs_secret_export": [_vp, _i64p, ctypes.c_size_t],
        "hs_pk_export": [_vp, _u64p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)],
        "hs_encode": [_vp, _f64p, _vp, ctypes.c_size_t, S, ctypes.c_double, _u64p],
        "hs_encode_encrypt": [_vp, _f64p, _vp, ctypes.c_size_t, S, ctypes.c_double, ctypes.c_uint64,
                              ctypes.POINTER(_vp)],
        "hs_encrypt_rows": [_vp, _u64p, S, ctypes.c_double, ctypes.c_uint64, ctypes.POINTER(_vp)],
        "hs_decrypt_decode": [_vp, _vp, _f64p, _vp, ctypes.c_size_t],
        "hs_ct_export": [_vp, _vp, _u64p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)],
        "hs_ct_import": [_vp, _u64p, S, S, ctypes.c_double, ctypes.POINTER(_vp)],
        "hs_ct_info": [_vp, ctypes.POINTER(S), ctypes.POINTER(S), ctypes.POINTER(ctypes.c_double)],
        "hs_ct_set_scale": [_vp, ctypes.c_double],
        "hs_add": [_vp, _vp, _vp, ctypes.POINTER(_vp)],
        "hs_sub": [_vp, _vp, _vp, ctypes.POINTER(_vp)],
        "hs_tensor": [_vp, _vp, _vp, ctypes.POINTER(_vp)],
        "hs_relinearize": [_vp, _vp, ctypes.POINTER(_vp)],
        "hs_rescale": [_vp, _vp, ctypes.POINTER(_vp)],
        "hs_mult_relin": [_vp, _vp, _vp, S, ctypes.POINTER(_vp)],
        "hs_mult_relin_noalloc": [_vp, _vp, _vp, S, ctypes.c_double, ctypes.c_double, S, _vp,
                                  ctypes.POINTER(ctypes.c_double)],
        "hs_rotate": [_vp, _vp, ctypes.c_int32, ctypes.POINTER(_vp)],
        "hs_rotate_hoisted": [_vp, _vp, ctypes.POINTER(ctypes.c_int32), ctypes.c_size_t, ctypes.POINTER(_vp)],
        "hs_rotate_batch": [_vp, ctypes.POINTER(_vp), ctypes.POINTER(ctypes.c_int32), ctypes.c_size_t,
                            ctypes.POINTER(_vp)],
        "hs_conjugate": [_vp, _vp, ctypes.POINTER(_vp)],
        "hs_mul_plain_rows": [_vp, _vp, _u64p, ctypes.c_double, S, ctypes.POINTER(_vp)],
        "hs_mul_int": [_vp, _vp, ctypes.c_int64, ctypes.POINTER(_vp)],
        "hs_add_const": [_vp, _vp, ctypes.c_double, ctypes.POINTER(_vp)],
        "hs_mod_drop": [_vp, _vp, S, ctypes.POINTER(_vp)],
        "hs_mod_raise": [_vp, _vp, S, ctypes.POINTER(_vp)],
        "hs_mul_monomial": [_vp, _vp, S, ctypes.POINTER(_vp)],
        "hs_dbg_ntt": [_vp, S, _u64p, ctypes.c_size_t, S],
        "hs_dbg_mul_rate": [_vp, ctypes.POINTER(ctypes.c_double)],
        "hs_dbg_minimax": [ctypes.c_double, ctypes.c_double, S, ctypes.c_double, ctypes.POINTER(ctypes.c_double)],
        "hs_dbg_ntt_time": [_vp, S, S, S, S, ctypes.POINTER(ctypes.c_double)],
        "hs_dbg_ring": [_vp, S, S, S, _u64p, ctypes.c_size_t, _u64p, ctypes.c_size_t,
                        ctypes.POINTER(ctypes.c_size_t)],
        "hs_ctx_memory": [_vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)],
        "hs_stream_create": [S, ctypes.POINTER(_vp)],
        "hs_stream_destroy": [_vp],
        "hs_ctx_trim": [_vp, ctypes.POINTER(ctypes.c_size_t)],
    }
    optional = {
        "hs_bootstrap": [_vp, _vp, ctypes.POINTER(_vp)],
        "hs_dbg_bootstrap_stage": [_vp, _vp, S, ctypes.POINTER(_vp)],
        "hs_prof_enable": [_vp, S],
        "hs_prof_collect": [_vp, ctypes.POINTER(ctypes.c_double), ctypes.c_size_t],
        "hs_softmax": [_vp, ctypes.POINTER(_vp), ctypes.c_size_t, ctypes.c_uint32, ctypes.c_double,
                       ctypes.POINTER(hs_softmax_opts), ctypes.POINTER(_vp)],
        "hs_softmax_jobs": [_vp, ctypes.POINTER(_vp), ctypes.c_size_t, ctypes.c_size_t, ctypes.c_uint32,
                            ctypes.c_double, ctypes.POINTER(hs_softmax_opts), ctypes.POINTER(_vp)],
        "hs_softmax_stats": [_vp, ctypes.POINTER(ctypes.c_double), ctypes.c_size_t],
        "hs_op_counts": [_vp, ctypes.POINTER(ctypes.c_double), ctypes.c_size_t, S],
        "hs_softmax_plan_create": [_vp, ctypes.POINTER(_vp), ctypes.c_size_t, ctypes.c_size_t, ctypes.c_uint32,
                                   ctypes.c_double, ctypes.POINTER(hs_softmax_opts), ctypes.POINTER(_vp)],
        "hs_softmax_plan_run": [_vp, ctypes.POINTER(_vp), ctypes.c_size_t, ctypes.POINTER(_vp)],
        "hs_softmax_plan_info": [_vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)],
        "hs_tune_enable": [S],
        "hs_tune_clear": [],
        "hs_tune_report": [ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)],
        "hs_tune_save": [ctypes.c_char_p],
        "hs_tune_load": [ctypes.c_char_p, ctypes.POINTER(S)],
        "hs_pack_softmax": [_f64p, ctypes.c_size_t, ctypes.c_uint32, ctypes.c_size_t, ctypes.c_double, _vp,
                            ctypes.POINTER(ctypes.c_size_t)],
        "hs_unpack_softmax": [_f64p, ctypes.c_size_t, ctypes.c_uint32, ctypes.c_size_t, _f64p],
    }
    for name, args in list(sig.items()) + list(optional.items()):
        if not hasattr(L, name):
            if name in sig:
                raise ImportError("libhs.so lacks %s" % name)
            continue
        f = getattr(L, name)
        f.argtypes = args
        f.restype = S
    L.hs_ct_destroy.argtypes = [_vp]
    L.hs_ct_destroy.restype = None
    L.hs_ctx_destroy.argtypes = [_vp]
    L.hs_ctx_destroy.restype = None
    if hasattr(L, "hs_softmax_plan_destroy"):
        L.hs_softmax_plan_destroy.argtypes = [_vp]
        L.hs_softmax_plan_destroy.restype = None
    _lib = L
    return L


def _check(st):
    if st != 0:
        raise HSError(st, lib().hs_last_error().decode())


def minimax(a, b, degree, e):
    """hs_dbg_minimax (host only): Chebyshev coefficients on [a, b] of the
    weighted minimax approximant of s^-e the Softmax uses."""
    c = (ctypes.c_double * (degree + 1))()
    _check(lib().hs_dbg_minimax(a, b, degree, e, c))
    return np.array(c[:], dtype=np.float64)


def stream_create(device=0):
    """A new HIP stream owned by the caller (hs_stream_create)."""
    st = _vp()
    _check(lib().hs_stream_create(device, ctypes.byref(st)))
    return st


def stream_destroy(stream):
    _check(lib().hs_stream_destroy(stream))


def current_stream():
    """HIP stream handle of torch's current stream on the current device."""
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Ciphertext:
    def __init__(self, ctx, handle):
        self.ctx = ctx
        self.h = handle

    def __del__(self):
        # after its context was closed the handle is left alone (its device
        # block went back with the context)
        if getattr(self, "h", None) and _lib is not None and getattr(self.ctx, "h", None):
            _lib.hs_ct_destroy(self.h)
            self.h = None

    @property
    def info(self):
        lv, nc, sc = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        _check(lib().hs_ct_info(self.h, ctypes.byref(lv), ctypes.byref(nc), ctypes.byref(sc)))
        return lv.value, nc.value, sc.value

    @property
    def level(self):
        return self.info[0]

    @property
    def scale(self):
        return self.info[2]

    def export(self):
        used = ctypes.c_size_t()
        _check(lib().hs_ct_export(self.ctx.h, self.h, np.zeros(1, np.uint64), 0, ctypes.byref(used)))
        out = np.zeros(used.value, dtype=np.uint64)
        _check(lib().hs_ct_export(self.ctx.h, self.h, out, out.size, ctypes.byref(used)))
        lv, nc, _ = self.info
        return out.reshape(nc, lv + 1, -1)


def tune_enable(on=True):
    """hs_tune_enable: time interchangeable kernels on the first launch of each shape."""
    _check(lib().hs_tune_enable(1 if on else 0))


def tune_clear():
    """hs_tune_clear: forget every decision (default kernels again)."""
    _check(lib().hs_tune_clear())


def tune_report():
    """Autotuner decisions: list of dicts {key, choice, us}."""
    import json
    used = ctypes.c_size_t()
    _check(lib().hs_tune_report(None, 0, ctypes.byref(used)))
    buf = ctypes.create_string_buffer(used.value)
    _check(lib().hs_tune_report(buf, used.value, ctypes.byref(used)))
    return [json.loads(l) for l in buf.value.decode().splitlines() if l.strip()]


def tune_save(path):
    _check(lib().hs_tune_save(str(path).encode()))


def tune_load(path):
    n = ctypes.c_int()
    _check(lib().hs_tune_load(str(path).encode(), ctypes.byref(n)))
    return n.value


class SoftmaxPlan:
    """A captured Softmax schedule (hs_softmax_plan_*); keeps its context alive."""

    def __init__(self, ctx, handle, m):
        self.ctx = ctx
        self.h = handle
        self.m = m

    def run(self, cts):
        if len(cts) != self.m:
            raise ValueError("plan takes %d ciphertexts" % self.m)
        arr = (_vp * self.m)(*[c.h for c in cts])
        out = (_vp * self.m)()
        _check(lib().hs_softmax_plan_run(self.h, arr, self.m, out))
        return [Ciphertext(self.ctx, _vp(out[i])) for i in range(self.m)]

    def info(self):
        """(graph nodes, arena bytes)"""
        a, b = ctypes.c_size_t(), ctypes.c_size_t()
        _check(lib().hs_softmax_plan_info(self.h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.hs_softmax_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)


class DeviceAllocator:
    """Allocator callbacks of a context (hs_ctx_create_ex): ``get(nbytes,
    stream)`` returns a device address or None, ``put(ptr, nbytes)`` takes it
    back.  ``live`` maps the addresses handed out to their sizes."""

    def __init__(self):
        self.live = {}
        self.alloc_cb = _ALLOC_FN(self._alloc)
        self.free_cb = _FREE_FN(self._free)

    def _alloc(self, nbytes, stream, user):
        try:
            p = self.get(int(nbytes), int(stream or 0))
        except Exception:           # no memory (or any failure): the library raises HS_E_OOM
            return None
        if p:
            self.live[int(p)] = int(nbytes)
        return p or None

    def _free(self, ptr, nbytes, user):
        self.live.pop(int(ptr), None)
        try:
            self.put(int(ptr), int(nbytes))
        except Exception:           # e.g. torch already torn down at interpreter exit
            pass

    def get(self, nbytes, stream):
        raise NotImplementedError

    def put(self, ptr, nbytes):
        raise NotImplementedError


class TorchAllocator(DeviceAllocator):
    """Device memory from torch's caching allocator, in stream order on the
    context's stream."""

    def __init__(self, device):
        super().__init__()
        self.device = device

    def get(self, nbytes, stream):
        import torch
        return torch.cuda.caching_allocator_alloc(nbytes, self.device, stream)

    def put(self, ptr, nbytes):
        import torch
        torch.cuda.caching_allocator_delete(ptr)


class Context:
    """One parameter set on one device.  ``params`` is a dict like the
    presets in ``synthetic.PRESETS``.  Device memory comes from ``allocator``:
    "torch" (torch's caching allocator, the default), None (the library's
    own hipMalloc) or a DeviceAllocator."""

    def __init__(self, params, device=0, stream=None, allocator="torch"):
        L = lib()
        self._keep = []
        qb = (ctypes.c_int * len(params["q_bits"]))(*params["q_bits"])
        pb = (ctypes.c_int * len(params["p_bits"]))(*params["p_bits"])
        self._keep += [qb, pb]
        boot = params.get("boot") or {}
        p = hs_params(
            log_n=params["logN"], n_q=len(params["q_bits"]), q_bits=qb, n_p=len(params["p_bits"]),
            p_bits=pb, digit=params["digit"], hamming=params["hamming"], sigma=params.get("sigma", 3.2),
            log_scale=params["log_scale"], user_top=params["user_top"],
            boot_cts_levels=boot.get("cts_levels", 0), boot_evalmod_levels=boot.get("evalmod_levels", 0),
            boot_stc_levels=boot.get("stc_levels", 0), boot_K=boot.get("K", 0),
            boot_double_angle=boot.get("double_angle", 0), boot_cos_degree=boot.get("cos_degree", 0),
            boot_log_scale=boot.get("log_boot_scale", 0))
        h = _vp()
        st = stream if stream is not None else None
        if isinstance(allocator, str) and allocator == "torch":
            allocator = TorchAllocator(device)
        self.allocator = allocator          # the callbacks must outlive the context
        if allocator is None:
            _check(L.hs_ctx_create(ctypes.byref(p), device, st, ctypes.byref(h)))
        else:
            _check(L.hs_ctx_create_ex(ctypes.byref(p), device, st, allocator.alloc_cb, allocator.free_cb, None,
                                      ctypes.byref(h)))
        self.h = h
        info = hs_ctx_info()
        _check(L.hs_ctx_get_info(h, ctypes.byref(info)))
        self.N = info.n
        self.slots = info.slots
        self.nq = info.n_q
        self.np = info.n_p
        self.L = info.top_level
        self.user_top = info.user_top
        self.dnum = info.dnum
        self.delta = float(2 ** params["log_scale"])

    def clone(self, stream=None):
        """hs_ctx_clone: a context on `stream` sharing this one's keys."""
        c = Context.__new__(Context)
        h = _vp()
        _check(lib().hs_ctx_clone(self.h, stream, ctypes.byref(h)))
        c.__dict__.update({k: v for k, v in self.__dict__.items() if k not in ("h",)})
        c.h = h
        c.parent = self            # the parent outlives its clones
        return c

    def close(self):
        """hs_ctx_destroy now (every device block back to the allocator);
        ciphertexts of this context must not be used afterwards."""
        if getattr(self, "h", None) and _lib is not None:
            _lib.hs_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def primes(self):
        out = np.zeros(self.nq + self.np, dtype=np.uint64)
        n = ctypes.c_size_t()
        _check(lib().hs_ctx_primes(self.h, out, out.size, ctypes.byref(n)))
        return [int(v) for v in out]

    def sync(self):
        _check(lib().hs_sync(self.h))

    def keygen(self, seed, rotations=(), conj=False):
        _check(lib().hs_keygen(self.h, seed))
        self.add_rotation_keys(rotations, conj)

    def add_rotation_keys(self, rotations=(), conj=False):
        arr = (ctypes.c_int32 * max(1, len(rotations)))(*rotations)
        _check(lib().hs_add_rotation_keys(self.h, arr, len(rotations), 1 if conj else 0))

    def key_export(self, key_id):
        used = ctypes.c_size_t()
        _check(lib().hs_key_export(self.h, key_id, np.zeros(1, np.uint64), 0, ctypes.byref(used)))
        out = np.zeros(used.value, dtype=np.uint64)
        _check(lib().hs_key_export(self.h, key_id, out, out.size, ctypes.byref(used)))
        return out.reshape(self.dnum, 2, self.nq + self.np, self.N)

    def secret(self):
        out = np.zeros(self.N, dtype=np.int64)
        _check(lib().hs_secret_export(self.h, out, out.size))
        return out

    def pk_export(self):
        used = ctypes.c_size_t()
        out = np.zeros(2 * self.nq * self.N, dtype=np.uint64)
        _check(lib().hs_pk_export(self.h, out, out.size, ctypes.byref(used)))
        return out.reshape(2, self.nq, self.N)

    @staticmethod
    def _slots(z):
        z = np.asarray(z)
        re = np.ascontiguousarray(z.real, dtype=np.float64)
        im = np.ascontiguousarray(z.imag, dtype=np.float64) if np.iscomplexobj(z) else None
        return re, im

    def encode(self, z, level, scale):
        re, im = self._slots(z)
        out = np.zeros((level + 1) * self.N, dtype=np.uint64)
        _check(lib().hs_encode(self.h, re, im.ctypes.data if im is not None else None, re.size, level, scale, out))
        return out.reshape(level + 1, self.N)

    def encrypt(self, z, level, scale, seed):
        re, im = self._slots(z)
        h = _vp()
        _check(lib().hs_encode_encrypt(self.h, re, im.ctypes.data if im is not None else None, re.size, level,
                                       scale, seed, ctypes.byref(h)))
        return Ciphertext(self, h)

    def encrypt_rows(self, pt, level, scale, seed):
        h = _vp()
        _check(lib().hs_encrypt_rows(self.h, np.ascontiguousarray(pt, dtype=np.uint64).reshape(-1), level, scale,
                                     seed, ctypes.byref(h)))
        return Ciphertext(self, h)

    def decrypt(self, ct):
        re = np.zeros(self.slots)
        im = np.zeros(self.slots)
        _check(lib().hs_decrypt_decode(self.h, ct.h, re, im.ctypes.data, self.slots))
        return re + 1j * im

    def import_ct(self, words, level, ncomp, scale):
        h = _vp()
        _check(lib().hs_ct_import(self.h, np.ascontiguousarray(words, dtype=np.uint64).reshape(-1), level, ncomp,
                                  scale, ctypes.byref(h)))
        return Ciphertext(self, h)

    def _op(self, name, *args):
        h = _vp()
        _check(getattr(lib(), name)(self.h, *args, ctypes.byref(h)))
        return Ciphertext(self, h)

    def add(self, a, b):
        return self._op("hs_add", a.h, b.h)

    def sub(self, a, b):
        return self._op("hs_sub", a.h, b.h)

    def tensor(self, a, b):
        return self._op("hs_tensor", a.h, b.h)

    def relinearize(self, d):
        return self._op("hs_relinearize", d.h)

    def rescale(self, a):
        return self._op("hs_rescale", a.h)

    def mult(self, a, b, rescale=True):
        return self._op("hs_mult_relin", a.h, b.h, 1 if rescale else 0)

    def mult_noalloc(self, a_ptr, b_ptr, level, scale_a, scale_b, out_ptr, rescale=True):
        """hs_mult_relin_noalloc on raw device buffers (integer addresses of
        [2][level+1][N] uint64 residues each; out receives the product's
        [2][level'+1][N]); returns the output scale.  Asynchronous on the
        context's stream."""
        sc = ctypes.c_double()
        _check(lib().hs_mult_relin_noalloc(self.h, _vp(a_ptr), _vp(b_ptr), level, scale_a, scale_b,
                                           1 if rescale else 0, _vp(out_ptr), ctypes.byref(sc)))
        return sc.value

    def rotate(self, a, r):
        return self._op("hs_rotate", a.h, r)

    def rotate_hoisted(self, a, rots):
        """hs_rotate_hoisted: rotations of `a` by every r in rots, one ModUp."""
        n = len(rots)
        rs = (ctypes.c_int32 * n)(*rots)
        out = (_vp * n)()
        _check(lib().hs_rotate_hoisted(self.h, a.h, rs, n, out))
        return [Ciphertext(self, _vp(out[i])) for i in range(n)]

    def rotate_batch(self, cts, rots):
        """hs_rotate_batch: cts[i] rotated by rots[i], one batched key switch."""
        n = len(cts)
        arr = (_vp * n)(*[c.h for c in cts])
        rs = (ctypes.c_int32 * n)(*rots)
        out = (_vp * n)()
        _check(lib().hs_rotate_batch(self.h, arr, rs, n, out))
        return [Ciphertext(self, _vp(out[i])) for i in range(n)]

    def conjugate(self, a):
        return self._op("hs_conjugate", a.h)

    def mul_plain_rows(self, a, pt, pt_scale, rescale=False):
        return self._op("hs_mul_plain_rows", a.h, np.ascontiguousarray(pt, dtype=np.uint64).reshape(-1),
                        pt_scale, 1 if rescale else 0)

    def mul_int(self, a, k):
        return self._op("hs_mul_int", a.h, int(k))

    def add_const(self, a, v):
        return self._op("hs_add_const", a.h, float(v))

    def mod_drop(self, a, level):
        return self._op("hs_mod_drop", a.h, level)

    def mod_raise(self, a, level):
        return self._op("hs_mod_raise", a.h, level)

    def mul_monomial(self, a, k):
        return self._op("hs_mul_monomial", a.h, k)

    def bootstrap(self, a):
        return self._op("hs_bootstrap", a.h)

    PROF_KINDS = ("ntt", "keyip", "conv", "tensor", "ew", "perm", "lift", "other")

    def prof_enable(self, on=True):
        _check(lib().hs_prof_enable(self.h, 1 if on else 0))

    def prof_collect(self):
        buf = (ctypes.c_double * 24)()
        _check(lib().hs_prof_collect(self.h, buf, 24))
        return {k: dict(launches=int(buf[3 * i]), ms=float(buf[3 * i + 1]), bytes=float(buf[3 * i + 2]))
                for i, k in enumerate(self.PROF_KINDS)}

    def bootstrap_stage(self, a, stage):
        return self._op("hs_dbg_bootstrap_stage", a.h, stage)

    def softmax(self, cts, n, M, variant=0, k=0, exp_degree=0, inv_degrees=(0, 0, 0), debug_stop=-1, jobs=1,
                power=0, newton_steps=0, mask_mode=0, approx=0, merge=0):
        """hs_softmax (jobs = 1) or hs_softmax_jobs over the packed ciphertexts
        `cts` (jobs consecutive groups of len(cts) / jobs); returns new handles.
        merge = 1: the jobs share one auxiliary ciphertext (version B)."""
        m = len(cts)
        arr = (_vp * m)(*[c.h for c in cts])
        out = (_vp * m)()
        o = hs_softmax_opts(variant=variant, k=k, exp_degree=exp_degree, inv_degree_first=inv_degrees[0],
                            inv_degree_mid=inv_degrees[1], inv_degree_last=inv_degrees[2], alpha=0.0,
                            power=power, debug_stop=debug_stop, newton_steps=newton_steps, mask_mode=mask_mode,
                            approx=approx, merge=merge)
        if jobs == 1:
            _check(lib().hs_softmax(self.h, arr, m, n, M, ctypes.byref(o), out))
        else:
            _check(lib().hs_softmax_jobs(self.h, arr, m, jobs, n, M, ctypes.byref(o), out))
        return [Ciphertext(self, _vp(out[i])) for i in range(m)]

    def softmax_plan(self, cts, n, M, variant=0, k=0, exp_degree=0, inv_degrees=(0, 0, 0), jobs=1, power=0,
                     newton_steps=0, mask_mode=0, approx=0, merge=0):
        """hs_softmax_plan_create: capture the schedule of softmax(cts, ...)
        once (after one eager warm-up run on `cts`) for replays on new inputs
        of the same shape, level and scale."""
        m = len(cts)
        arr = (_vp * m)(*[c.h for c in cts])
        o = hs_softmax_opts(variant=variant, k=k, exp_degree=exp_degree, inv_degree_first=inv_degrees[0],
                            inv_degree_mid=inv_degrees[1], inv_degree_last=inv_degrees[2], alpha=0.0,
                            power=power, debug_stop=-1, newton_steps=newton_steps, mask_mode=mask_mode,
                            approx=approx, merge=merge)
        h = _vp()
        _check(lib().hs_softmax_plan_create(self.h, arr, m, jobs, n, M, ctypes.byref(o), ctypes.byref(h)))
        return SoftmaxPlan(self, h, m)

    OP_KINDS = ("keyswitch", "tensor", "rescale", "ptmul", "add")

    def op_counts(self, clear=True):
        """hs_op_counts: {kind: {level: ciphertext equivalents}} since the last
        clear (eager launches only)."""
        buf = (ctypes.c_double * (5 * 64))()
        _check(lib().hs_op_counts(self.h, buf, 5 * 64, 1 if clear else 0))
        return {k: {l: buf[i * 64 + l] for l in range(64) if buf[i * 64 + l]} for i, k in enumerate(self.OP_KINDS)}

    def softmax_stats(self):
        buf = (ctypes.c_double * 4)()
        _check(lib().hs_softmax_stats(self.h, buf, 4))
        return dict(k=int(buf[0]), bootstraps=int(buf[1]), levels_left=int(buf[2]), ms=float(buf[3]))

    def memory(self):
        """(bytes in use, bytes reserved) of the context's device arena."""
        a, b = ctypes.c_size_t(), ctypes.c_size_t()
        _check(lib().hs_ctx_memory(self.h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def trim(self):
        """Return unused arena chunks to the device; bytes released."""
        r = ctypes.c_size_t()
        _check(lib().hs_ctx_trim(self.h, ctypes.byref(r)))
        return r.value

    def ntt_time(self, groups, level, reps=20, inverse=False):
        """hs_dbg_ntt_time: average microseconds per NTT launch over `groups`
        groups of level+1 rows."""
        us = ctypes.c_double()
        _check(lib().hs_dbg_ntt_time(self.h, groups, level, reps, 1 if inverse else 0, ctypes.byref(us)))
        return us.value

    def mul_rate(self):
        """Measured v_mad_u64_u32 throughput of the device (10^12 ops/s)."""
        t = ctypes.c_double()
        _check(lib().hs_dbg_mul_rate(self.h, ctypes.byref(t)))
        return t.value

    RING_OPS = {"ntt": 0, "intt": 1, "modup": 2, "moddown": 3, "auto": 4, "rescale": 5, "tensor": 6}

    def ring(self, op, rows, level, arg=0):
        """hs_dbg_ring: one raw ring operation on host rows (see include/hs.h)."""
        x = np.ascontiguousarray(rows, dtype=np.uint64).reshape(-1)
        code = self.RING_OPS[op]
        used = ctypes.c_size_t()
        _check(lib().hs_dbg_ring(self.h, code, level, arg, x, x.size, np.zeros(1, np.uint64), 0,
                                 ctypes.byref(used)))
        out = np.zeros(used.value, dtype=np.uint64)
        _check(lib().hs_dbg_ring(self.h, code, level, arg, x, x.size, out, out.size, ctypes.byref(used)))
        return out.reshape(-1, self.N)

    def ntt(self, rows, prime, inverse=False):
        x = np.ascontiguousarray(rows, dtype=np.uint64).copy()
        _check(lib().hs_dbg_ntt(self.h, prime, x.reshape(-1), x.size // self.N, 1 if inverse else 0))
        return x


def pack_softmax(logits, slots, M):
    """hs_pack_softmax: (L, n) logits -> (m, slots) slot vectors."""
    logits = np.ascontiguousarray(logits, dtype=np.float64)
    L, n = logits.shape
    m = ctypes.c_size_t()
    _check(lib().hs_pack_softmax(logits.reshape(-1), L, n, slots, M, None, ctypes.byref(m)))
    out = np.zeros((m.value, slots))
    _check(lib().hs_pack_softmax(logits.reshape(-1), L, n, slots, M, out.ctypes.data, ctypes.byref(m)))
    return out


def unpack_softmax(slot_vecs, n):
    slot_vecs = np.ascontiguousarray(slot_vecs, dtype=np.float64)
    m, slots = slot_vecs.shape
    n2 = 1 << (int(n) - 1).bit_length()          # packed as the next power of two
    out = np.zeros((m * slots // n2, n))
    _check(lib().hs_unpack_softmax(slot_vecs.reshape(-1), m, n, slots, out))
    return out
