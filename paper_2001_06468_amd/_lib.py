"""ctypes declarations of the libnrs C ABI (include/nrs.h).  Marshalling only."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnrs.so")

NRS_OK = 0
NRS_E_ARG = -1
NRS_E_HIP = -2
NRS_E_WORKSPACE = -3
NRS_E_SINGULAR = -4
NRS_E_NOT_CONVERGED = -5
NRS_E_NONFINITE = -6
NRS_E_UNSUPPORTED = -7

NRS_FP64_LU = 0
NRS_FP32_IR = 1
NRS_FP32_GEPP_IR = 2
NRS_GMRES = 3
NRS_FP32_GMRES_IR = 4
NRS_BF16_GMRES_IR = 5
NRS_GMRES_BLOCK = 6

NRS_PRECOND_EXACT = 0
NRS_PRECOND_MODEL = 1
NRS_BLOCK_MAX_HARMONICS = 16

NRS_WARM_NONE = 0
NRS_WARM_PREVIOUS = 1
NRS_WARM_MODEL = 2
NRS_MLP_HIDDEN = 64
NRS_MLP_MAX_POINTS = 256
NRS_NOALLOC_MAX_N = 65536

_p = C.c_void_p
_i64 = C.c_int64
_i32 = C.c_int32


class NrsScene(C.Structure):
    _fields_ = [("N", _i64), ("Q", _i64), ("M", _i32), ("P", _i32),
                ("xi", _p), ("body", _p), ("part", _p), ("s", _p), ("ufix", _p),
                ("Xi", _p), ("bodyX", _p), ("partX", _p), ("sX", _p), ("w0", _p),
                ("wave", _p)]


class NrsProblem(C.Structure):
    _fields_ = [("N", _i64), ("Q", _i64), ("M", _i32),
                ("x", _p), ("X", _p), ("w", _p), ("nu", _p), ("body", _p), ("Y", _p),
                ("eps", C.c_double), ("mu", C.c_double)]


class NrsOptions(C.Structure):
    _fields_ = [("method", _i32), ("max_refine", _i32), ("tol", C.c_double),
                ("gmres_restart", _i32), ("gmres_max_iter", _i32), ("no_fallback", _i32),
                ("x_init", _p), ("warm_start", _i32), ("model_theta", _p),
                ("model_scales", C.c_double * 3), ("body_off", _p), ("x_init_complete", _i32),
                ("graph", _i32), ("reuse_stage_factors", _i32), ("equilibrate", _i32),
                ("precond", _i32), ("precond_harmonics", _i32), ("precond_nb", _i32),
                ("precond_model", _p), ("precond_phase", _p), ("ir_queue", _i32)]


class NrsInfo(C.Structure):
    _fields_ = [("method_used", _i32), ("fell_back", _i32), ("iterations", _i32),
                ("singular", _i32), ("backward_error", C.c_double), ("correction", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class NrsDopriStats(C.Structure):
    _fields_ = [("accepted", _i32), ("rejected", _i32), ("solves", _i32), ("fell_back", _i32),
                ("t", C.c_double), ("h", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class NrsTuneResult(C.Structure):
    _fields_ = [("size_class", _i32), ("block32", _i32), ("strip32", _i32), ("block64", _i32),
                ("strip64", _i32), ("ms32", C.c_float), ("ms64", C.c_float),
                ("default_ms32", C.c_float), ("default_ms64", C.c_float)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# name -> (restype, argtypes); every function declared in include/nrs.h
PROTOTYPES = {
    "nrs_create": (_i32, [C.POINTER(_p), C.c_int, _p]),
    "nrs_destroy": (_i32, [_p]),
    "nrs_set_stream": (_i32, [_p, _p]),
    "nrs_status_string": (C.c_char_p, [_i32]),
    "nrs_last_error": (C.c_char_p, [_p]),
    "nrs_version": (C.c_char_p, []),
    "nrs_geometry": (_i32, [_p, C.POINTER(NrsScene), C.c_double, _p, _p, _p, _p, _p]),
    "nrs_nearest": (_i32, [_p, _i64, _p, _i32, _p, _i64, _p, _p, _p]),
    "nrs_workspace_size": (_i32, [_p, _i64, _i64, _i32, _i32, C.POINTER(C.c_size_t)]),
    "nrs_assemble": (_i32, [_p, C.POINTER(NrsProblem), _i32, _p, _i64, _p, C.c_size_t]),
    "nrs_apply": (_i32, [_p, C.POINTER(NrsProblem), _p, _p, _p, C.c_size_t]),
    "nrs_solve": (_i32, [_p, C.POINTER(NrsProblem), _p, _p, C.POINTER(NrsOptions), _p,
                         C.c_size_t, _p, C.POINTER(NrsInfo)]),
    "nrs_query_info": (_i32, [_p, _p, C.POINTER(NrsInfo)]),
    "nrs_solve_batched_workspace_size": (_i32, [_p, _i32, C.POINTER(NrsProblem), _i32,
                                                C.POINTER(C.c_size_t)]),
    "nrs_solve_batched": (_i32, [_p, _i32, C.POINTER(NrsProblem), C.POINTER(_p), C.POINTER(_p),
                                 C.POINTER(NrsOptions), _p, C.c_size_t, C.POINTER(_p),
                                 C.POINTER(NrsInfo)]),
    "nrs_lu_factor_workspace_size": (_i32, [_p, _i64, _i32, C.POINTER(C.c_size_t)]),
    "nrs_lu_factor": (_i32, [_p, _i64, _i32, _i32, _p, _i64, _p, _p, _p, _p, C.c_size_t]),
    "nrs_lu_solve_workspace_size": (_i32, [_p, _i64, C.POINTER(C.c_size_t)]),
    "nrs_lu_solve": (_i32, [_p, _i64, _i32, _i32, _p, _i64, _p, _p, _p, _p, C.c_size_t]),
    "nrs_lu_query": (_i32, [_p, _p, C.POINTER(_i32)]),
    "nrs_lu_solve_noalloc": (_i32, [_p, _i64, _i32, _i32, _p, _i64, _p, _p, _p]),
    "nrs_equilibrate": (_i32, [_p, _i64, _p, _i64, _p, _p, _p, C.c_size_t]),
    "nrs_autotune": (_i32, [_p, C.POINTER(NrsProblem), _p, C.c_size_t, C.POINTER(NrsTuneResult)]),
    "nrs_autotune_clear": (_i32, [_p]),
    "nrs_block_limit": (_i32, [_p, C.POINTER(_i32)]),
    "nrs_block_invert": (_i32, [_p, _i32, _i32, _p, _p]),
    "nrs_block_model_fit": (_i32, [_p, _i32, _i32, _i32, _p, _p]),
    "nrs_block_model_eval": (_i32, [_p, _i32, _i32, _p, _i32, _p, _p]),
    "nrs_mlp_param_count": (_i64, []),
    "nrs_mlp_body_offsets": (_i32, [_p, _i64, _p, _i32, _p]),
    "nrs_mlp_features": (_i32, [_p, _i64, _p, _p, _p, _p, _i32, _p, _p]),
    "nrs_mlp_forward": (_i32, [_p, _p, _i64, _i32, _p, _p, _i32, _p, _p, _p]),
    "nrs_mlp_grad_workspace_size": (_i32, [_i32, C.POINTER(C.c_size_t)]),
    "nrs_mlp_grad": (_i32, [_p, _p, _i64, _i32, _p, _p, _i32, _p, _p, _p, _p, _p, C.c_size_t]),
    "nrs_adam_step": (_i32, [_p, _i64, _p, _p, _p, _p, _i32, C.c_float, C.c_float, C.c_float,
                             C.c_float]),
    "nrs_mlp_targets": (_i32, [_p, _i64, _i32, _p, _p, _p, C.POINTER(C.c_double), _p, _p]),
    "nrs_mlp_warm_start_workspace_size": (_i32, [_i64, _i32, C.POINTER(C.c_size_t)]),
    "nrs_mlp_warm_start": (_i32, [_p, _p, C.POINTER(C.c_double), _i64, _i32, _p, _p, _p, _p, _p,
                                  _p, _p, _p, C.c_size_t]),
    "nrs_mlp_status": (_i32, [_p, C.POINTER(_i32)]),
    "nrs_rk4_workspace_size": (_i32, [_p, C.POINTER(NrsScene), _i32, C.POINTER(C.c_size_t)]),
    "nrs_rk4_step": (_i32, [_p, C.POINTER(NrsScene), _i32, _p, _p, C.c_double, C.c_double, _p,
                            _p, C.c_double, C.c_double, C.POINTER(NrsOptions), _p, C.c_size_t]),
    "nrs_dopri5_workspace_size": (_i32, [_p, C.POINTER(NrsScene), _i32, C.POINTER(C.c_size_t)]),
    "nrs_dopri5_integrate": (_i32, [_p, C.POINTER(NrsScene), _i32, _p, _p, C.c_double, C.c_double,
                                    _p, _p, C.c_double, C.c_double, C.POINTER(C.c_double),
                                    C.c_double, C.c_double, C.POINTER(NrsOptions), _i32,
                                    C.POINTER(NrsDopriStats), _p, C.c_size_t]),
    "nrs_field_workspace_size": (_i32, [_p, _i64, _i64, C.POINTER(C.c_size_t)]),
    "nrs_field_velocity": (_i32, [_p, C.POINTER(NrsProblem), _p, _i64, _p, _p, _p, C.c_size_t]),
    "nrs_tracer_rk4_step": (_i32, [_p, C.POINTER(NrsProblem), C.POINTER(_p), _i64, _p,
                                   C.c_double, _p, C.c_size_t]),
    "nrs_rk4_tracers_workspace_size": (_i32, [_p, C.POINTER(NrsScene), _i32, _i64,
                                              C.POINTER(C.c_size_t)]),
    "nrs_rk4_step_tracers": (_i32, [_p, C.POINTER(NrsScene), _i32, _p, _p, C.c_double,
                                    C.c_double, _p, _p, C.c_double, C.c_double,
                                    C.POINTER(NrsOptions), _i64, _p, _p, C.c_size_t]),
}

_LIB = None


def load(path: str = LIB_PATH):
    """Load libnrs.so; raises ImportError if the HIP library has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise ImportError(f"{path} not found: build the HIP library first "
                          "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = C.CDLL(path)
    for name, (res, args) in PROTOTYPES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib
