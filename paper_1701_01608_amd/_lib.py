"""ctypes declarations of the libfks C ABI (include/fks.h).  Marshalling only."""

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfks.so")

FKS_HARD_SPHERES = 0
FKS_VHS = 1
FKS_F64 = 0
FKS_F32 = 1
FKS_CONSERVE = 1
FKS_ALLOW_OVERLAP = 2
FKS_SUR_CENTER = 1

STATUS = {0: "FKS_OK", -1: "FKS_E_ARG", -2: "FKS_E_UNSUPPORTED", -3: "FKS_E_WORKSPACE",
          -4: "FKS_E_DEVICE", -5: "FKS_E_STATE"}


class FKSError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class CollideDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("kernel", ctypes.c_int32), ("L", ctypes.c_double),
                ("R", ctypes.c_double), ("alpha", ctypes.c_double), ("C", ctypes.c_double),
                ("a1", ctypes.c_int32), ("a2", ctypes.c_int32), ("n_radial", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("flags", ctypes.c_uint32), ("reserved", ctypes.c_int32)]


class StepOpts(ctypes.Structure):
    _fields_ = [("collision", ctypes.c_int32), ("integrator", ctypes.c_int32), ("nu", ctypes.c_double),
                ("nu_density", ctypes.c_int32), ("reserved", ctypes.c_int32), ("mu", ctypes.c_double),
                ("d_cons", ctypes.c_void_p), ("d_prim", ctypes.c_void_p), ("d_moments", ctypes.c_void_p),
                ("q_last", ctypes.c_void_p)]


FKS_COLL_BOLTZMANN, FKS_COLL_BGK = 0, 1
FKS_INT_EULER, FKS_INT_EXP = 0, 1


class ProfileStats(ctypes.Structure):
    _fields_ = [("total_ms", ctypes.c_double * 8), ("launches", ctypes.c_int64 * 8)]


PROFILE_SLOTS = ("forward", "slab", "finish", "xport_advance", "xport_roll", "moments")

_lib = None

# name: (restype, argtypes)
_VP = ctypes.c_void_p
_SIGS = {
    "fks_plan_create": (ctypes.c_int, [ctypes.POINTER(CollideDesc), ctypes.c_int64, ctypes.POINTER(_VP)]),
    "fks_plan_sizes": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]),
    "fks_plan_info": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "fks_plan_bind": (ctypes.c_int, [_VP, _VP, ctypes.c_size_t, _VP, ctypes.c_size_t, _VP]),
    "fks_collide": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int64, _VP]),
    "fks_collide_noalloc": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int64, _VP]),
    "fks_relax": (ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.c_double, ctypes.c_int64, _VP, _VP]),
    "fks_moments": (ctypes.c_int, [_VP, _VP, ctypes.c_int64, _VP, _VP]),
    "fks_noneq": (ctypes.c_int, [_VP, _VP, ctypes.c_int64, _VP, _VP]),
    "fks_heun": (ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.c_double, ctypes.c_int32, ctypes.c_int64, _VP]),
    "fks_graph_begin": (ctypes.c_int, [_VP]),
    "fks_graph_end": (ctypes.c_int, [_VP, ctypes.POINTER(_VP)]),
    "fks_graph_launch": (ctypes.c_int, [_VP, _VP]),
    "fks_graph_destroy": (None, [_VP]),
    "fks_collide_grouped": (ctypes.c_int, [ctypes.POINTER(_VP), ctypes.c_int32, ctypes.POINTER(_VP),
                                           ctypes.POINTER(_VP), ctypes.POINTER(ctypes.c_int64), _VP]),
    "fks_plan_destroy": (None, [_VP]),
    "fks_plan_schedule": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "fks_plan_set_schedule": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int32]),
    "fks_plan_set_term_groups": (ctypes.c_int, [_VP, ctypes.c_int32]),
    "fks_plan_get_term_groups": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "fks_plan_autotune": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int64, ctypes.c_char_p, _VP]),
    "fks_xport_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_double, ctypes.POINTER(_VP)]),
    "fks_xport_sizes": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_size_t)]),
    "fks_xport_bind": (ctypes.c_int, [_VP, _VP, ctypes.c_size_t, _VP]),
    "fks_transport": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int32, ctypes.c_double, _VP]),
    "fks_transport_ex": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, _VP]),
    "fks_step": (ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.c_double, ctypes.c_int32, _VP, _VP]),
    "fks_step_ex": (ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.c_double, ctypes.c_int32, ctypes.POINTER(StepOpts),
                                   _VP]),
    "fks_xport_destroy": (None, [_VP]),
    "fks_sur_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                      ctypes.c_float, ctypes.c_uint32, ctypes.POINTER(_VP)]),
    "fks_sur_sizes": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t),
                                     ctypes.POINTER(ctypes.c_int64)]),
    "fks_sur_bind": (ctypes.c_int, [_VP, _VP, ctypes.c_size_t, _VP, ctypes.c_size_t, _VP]),
    "fks_sur_set_params": (ctypes.c_int, [_VP, _VP, _VP]),
    "fks_sur_get": (ctypes.c_int, [_VP, ctypes.c_int32, _VP, _VP]),
    "fks_sur_features": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _VP, ctypes.c_int64, _VP]),
    "fks_sur_targets": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _VP, ctypes.c_int64, _VP]),
    "fks_sur_forward": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int64, _VP]),
    "fks_sur_train_step": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int64, ctypes.c_float, ctypes.c_int32, _VP,
                                          _VP]),
    "fks_sur_infer": (ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.c_int64, ctypes.c_double,
                                     ctypes.POINTER(ctypes.c_int64), _VP, _VP]),
    "fks_sur_infer_ranked": (ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.c_int64, ctypes.c_double,
                                     ctypes.POINTER(ctypes.c_int64), _VP, _VP]),
    "fks_sur_destroy": (None, [_VP]),
    "fks_profile_start": (ctypes.c_int, []),
    "fks_profile_stop": (ctypes.c_int, [ctypes.POINTER(ProfileStats)]),
    "fks_last_error": (ctypes.c_char_p, []),
    "fks_version": (ctypes.c_char_p, []),
}

EXPORTS = tuple(_SIGS)


def lib():
    """The loaded libfks; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1701_01608_amd.build` (no CPU fallback exists)")
        h = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(h, name)
            fn.restype = res
            fn.argtypes = args
        _lib = h
    return _lib


def check(status):
    if status != 0:
        msg = lib().fks_last_error()
        raise FKSError(status, msg.decode() if msg else "")
    return status
