"""ctypes declarations of the C ABI in include/dnslab.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os
from ctypes import CFUNCTYPE, POINTER, c_char_p, c_double, c_int, c_int32, c_int64, c_size_t, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdnslab.so")

DNSLAB_OK = 0
ERRORS = {
    -1: "DNSLAB_EINVAL", -2: "DNSLAB_ENOMEM", -3: "DNSLAB_EUNSUPPORTED", -4: "DNSLAB_EHIP",
    -5: "DNSLAB_ESTATE", -6: "DNSLAB_EAGAIN", -7: "DNSLAB_ENONFINITE",
}
FP64, FP32_REFINE = 0, 1

# Every symbol the header declares; the CPU tests check that the library exports them.
EXPORTS = [
    "dnslab_workspace_bytes", "dnslab_init", "dnslab_step", "dnslab_read_diags", "dnslab_poisson",
    "dnslab_poisson_noalloc",
    "dnslab_project", "dnslab_scalar_step", "dnslab_momentum_rhs", "dnslab_scalar_rhs",
    "dnslab_filter", "dnslab_set_time", "dnslab_destroy", "dnslab_last_error",
    "dnslab_profile_enable", "dnslab_profile_read", "dnslab_set_graph_steps", "dnslab_set_overlap", "dnslab_set_stage_pairs", "dnslab_set_fft_pipeline", "dnslab_pool_set_graph",
    "dnslab_particles_step", "dnslab_particles_sort", "dnslab_co2_histogram", "dnslab_accumulate", "dnslab_body_force",
    "dnslab_pool_create", "dnslab_pool_admit", "dnslab_pool_step", "dnslab_pool_query",
    "dnslab_pool_read_field", "dnslab_pool_release", "dnslab_pool_usage", "dnslab_pool_last_error",
    "dnslab_pool_destroy",
]


# Allocator callbacks of dnslab_params / dnslab_pool_create.
ALLOC_FN = CFUNCTYPE(c_void_p, c_size_t, c_void_p)
FREE_FN = CFUNCTYPE(None, c_void_p, c_void_p)


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", c_int32), ("ny", c_int32), ("nz", c_int32),
        ("lx", c_double), ("ly", c_double), ("lz", c_double),
        ("nu", c_double), ("alpha_c", c_double), ("tau_f", c_double),
        ("body", c_double * 3),
        ("cfl", c_double), ("dt_fixed", c_double), ("u_ref", c_double),
        ("n_piter", c_int32), ("filter", c_int32), ("precision", c_int32),
        ("stream", c_void_p),
        ("project_each_stage", c_int32),
        ("alloc", ALLOC_FN), ("free_", FREE_FN), ("alloc_user", c_void_p),
    ]


class Diag(ctypes.Structure):
    _fields_ = [
        ("t", c_double), ("dt", c_double), ("ke", c_double), ("div_l2", c_double),
        ("co2_mass", c_double), ("co2_room_mean", c_double), ("cfl_max", c_double),
        ("step", c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ParticleParams(ctypes.Structure):
    _fields_ = [("rho_p", c_double), ("rho_f", c_double), ("g", c_double * 3)]


class DnslabError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load():
    """Load libdnslab.so from the package directory; fail loudly if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2204_02107_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P, V = POINTER, c_void_p
    sig = {
        "dnslab_workspace_bytes": (c_int, [P(Params), P(c_size_t)]),
        "dnslab_init": (c_int, [P(Params), V, c_int64, V, V, V, V, V, V, V, V, V, V, P(V)]),
        "dnslab_step": (c_int, [V, c_int32, P(Diag)]),
        "dnslab_read_diags": (c_int, [V, c_int32, P(Diag)]),
        "dnslab_poisson": (c_int, [V, V, V]),
        "dnslab_poisson_noalloc": (c_int, [P(Params), V, V]),
        "dnslab_project": (c_int, [V, V, V, V]),
        "dnslab_scalar_step": (c_int, [V, c_double]),
        "dnslab_momentum_rhs": (c_int, [V, V, V, V, V, V, V]),
        "dnslab_scalar_rhs": (c_int, [V, V, V, V, V, V]),
        "dnslab_filter": (c_int, [V, V, V]),
        "dnslab_set_time": (c_int, [V, c_double, c_int64]),
        "dnslab_destroy": (None, [V]),
        "dnslab_last_error": (c_char_p, [V]),
        "dnslab_profile_enable": (c_int, [V, c_char_p]),
        "dnslab_profile_read": (c_int, [V, P(c_double), P(c_int64)]),
        "dnslab_set_graph_steps": (c_int, [V, c_int32]),
        "dnslab_set_overlap": (c_int, [V, c_int32]),
        "dnslab_set_stage_pairs": (c_int, [V, c_int32]),
        "dnslab_set_fft_pipeline": (c_int, [V, c_int32]),
        "dnslab_particles_step": (c_int, [V, c_int64, V, V, V, P(ParticleParams), c_double]),
        "dnslab_particles_sort": (c_int, [V, c_int64, V, V, V]),
        "dnslab_co2_histogram": (c_int, [V, c_int32, c_double, c_double, V]),
        "dnslab_accumulate": (c_int, [V, V]),
        "dnslab_body_force": (c_int, [V, P(c_int32), V]),
        "dnslab_pool_set_graph": (c_int, [V, c_int32]),
        "dnslab_pool_create": (c_int, [c_size_t, c_int32, V, ALLOC_FN, FREE_FN, V, P(V)]),
        "dnslab_pool_admit": (c_int, [V, P(Params), c_int64, V, c_int64, V, V, V, V, V, V, V, V, V, V,
                                      P(c_int32)]),
        "dnslab_pool_step": (c_int, [V, c_int32]),
        "dnslab_pool_query": (c_int, [V, c_int32, P(Diag), P(c_int64), P(c_int32)]),
        "dnslab_pool_read_field": (c_int, [V, c_int32, c_int32, V]),
        "dnslab_pool_release": (c_int, [V, c_int32]),
        "dnslab_pool_usage": (c_int, [V, P(c_size_t), P(c_int32), P(c_int32)]),
        "dnslab_pool_last_error": (c_char_p, [V]),
        "dnslab_pool_destroy": (None, [V]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(rc, ctx=None):
    if rc != DNSLAB_OK:
        msg = load().dnslab_last_error(ctx)
        raise DnslabError(rc, msg.decode() if msg else "")
    return rc


def check_pool(rc, pool=None):
    if rc != DNSLAB_OK:
        msg = load().dnslab_pool_last_error(pool)
        raise DnslabError(rc, msg.decode() if msg else "")
    return rc


# ---------------------------------------------------------------------------
# Device memory for the library from PyTorch's caching allocator: the library
# calls these back (on the calling thread) for its workspace and releases the
# blocks after synchronising the streams that used them.
_TORCH_USERS = {}     # key -> (device index, stream handle)
_TORCH_HELD = {}      # key -> {pointer: bytes requested} of the blocks not yet freed


def _torch_alloc(nbytes, user):
    try:
        import torch
        key = int(user or 0)
        dev, stream = _TORCH_USERS[key]
        ptr = torch.cuda.caching_allocator_alloc(int(nbytes), device=dev, stream=stream)
        _TORCH_HELD.setdefault(key, {})[int(ptr)] = int(nbytes)
        return ptr
    except Exception:
        return None


def _torch_free(ptr, user):
    try:
        import torch
        _TORCH_HELD.get(int(user or 0), {}).pop(int(ptr), None)
        torch.cuda.caching_allocator_delete(int(ptr))
    except Exception:
        pass


TORCH_ALLOC = ALLOC_FN(_torch_alloc)     # kept alive for the life of the module
TORCH_FREE = FREE_FN(_torch_free)


class TorchAllocator:
    """(alloc, free_, alloc_user) for one device and stream."""

    _next = 1

    def __init__(self, device_index: int, stream_handle: int):
        self.key = TorchAllocator._next
        TorchAllocator._next += 1
        _TORCH_USERS[self.key] = (int(device_index), int(stream_handle))
        self.user = c_void_p(self.key)

    def fill(self, params):
        params.alloc = TORCH_ALLOC
        params.free_ = TORCH_FREE
        params.alloc_user = self.user
        return params

    def triple(self):
        return TORCH_ALLOC, TORCH_FREE, self.user

    def bytes_held(self) -> int:
        """Bytes the library has requested through this allocator and not
        freed yet (torch's own figure rounds each block up)."""
        return sum(_TORCH_HELD.get(self.key, {}).values())

    def close(self):
        _TORCH_USERS.pop(self.key, None)
        _TORCH_HELD.pop(self.key, None)
