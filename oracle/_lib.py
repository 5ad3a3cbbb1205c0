"""ctypes loader for the ring oracle's C core (``oracle/ring.c``).

TEST INFRASTRUCTURE ONLY: the oracle is imported by ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py``; the
product library never touches it.

The shared object is compiled with plain ``gcc -O2`` on first use (or by
``build_oracle()``), in-tree, next to the source.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ring.c")
_SO = os.path.join(_HERE, "_oracle_ring.so")

_u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_u64 = ctypes.c_uint64


def build_oracle(force=False):
    """Compile ring.c into _oracle_ring.so with gcc (single-threaded, -O2)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", _SRC, "-o", tmp])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        build_oracle()
        L = ctypes.CDLL(_SO)
        L.or_powmod.restype = _u64
        L.or_powmod.argtypes = [_u64, _u64, _u64]
        L.or_invmod.restype = _u64
        L.or_invmod.argtypes = [_u64, _u64]
        L.or_psi_tables.argtypes = [_u64, _u64, _u64, _u64p, _u64p]
        L.or_ntt_definition.argtypes = [_u64p, _u64p, _u64, _u64, _u64]
        L.or_ntt_fwd.argtypes = [_u64p, _u64, _u64, _u64p]
        L.or_ntt_inv.argtypes = [_u64p, _u64, _u64, _u64p]
        L.or_negacyclic_mul.argtypes = [_u64p, _u64p, _u64p, _u64, _u64]
        for name in ("or_vec_mul", "or_vec_add", "or_vec_sub"):
            getattr(L, name).argtypes = [_u64p, _u64p, _u64p, _u64, _u64]
        L.or_vec_scalar_mul.argtypes = [_u64p, _u64, _u64p, _u64, _u64]
        L.or_base_convert.argtypes = [_u64p, _u64p, ctypes.c_int, _u64p, _u64p, ctypes.c_int, _u64]
        L.or_base_convert_centered.argtypes = [_u64p, _u64p, ctypes.c_int, _u64p, _u64p, ctypes.c_int, _u64]
        L.or_automorph_perm.argtypes = [_u64, _u64, _u64p]
        L.or_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
        L.or_draw_block.argtypes = [_u64, _u64, _u64, _u32p]
        L.or_sample_uniform.argtypes = [_u64, _u64, _u64, _u64, _u64p]
        L.or_sample_ternary.argtypes = [_u64, _u64, _u64, _i64p]
        L.or_sample_sparse_ternary.argtypes = [_u64, _u64, _u64, _u64, _i64p]
        L.or_sample_cdt.argtypes = [_u64, _u64, _u64, _u64p, ctypes.c_int, _i64p]
        _lib = L
    return _lib
