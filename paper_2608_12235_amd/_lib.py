"""ctypes view of librcp.so (include/rcp.h).  Argument marshalling only.

Loading fails loudly when the HIP library has not been built: there is no
CPU fallback for any entry point.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librcp.so")
MAX_RUNGS = 16

RCP_OK, RCP_EINVAL, RCP_EBOX, RCP_ENOMEM, RCP_EDEVICE = 0, -1, -2, -3, -4
RCP_ENOTCONV, RCP_ENONFINITE, RCP_EPLACE, RCP_ESTATE = -5, -6, -7, -8
RCP_INIT_NONE, RCP_INIT_RSA, RCP_INIT_UNIFORM, RCP_INIT_RSA_DEVICE = 0, 1, 2, 3
RCP_PLACE_WINDOW = 65536

ERRNAMES = {0: "RCP_OK", -1: "RCP_EINVAL", -2: "RCP_EBOX", -3: "RCP_ENOMEM",
            -4: "RCP_EDEVICE", -5: "RCP_ENOTCONV", -6: "RCP_ENONFINITE",
            -7: "RCP_EPLACE", -8: "RCP_ESTATE"}


class RcpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (ERRNAMES.get(code, "?"), code, msg))
        self.code = code


class Params(C.Structure):
    _fields_ = [("size", C.c_uint32), ("beta1", C.c_double), ("beta2", C.c_double),
                ("eps_x", C.c_double), ("eps_k", C.c_double), ("skin_s", C.c_double),
                ("skin_g", C.c_double), ("level_ratio_pow2", C.c_int32)]


class Tuning(C.Structure):
    _fields_ = [("size", C.c_uint32), ("graph_iters", C.c_int32), ("xcd_remap", C.c_int32),
                ("fused_tail", C.c_int32), ("variant", C.c_int32), ("row_cost", C.c_int32),
                ("item_work", C.c_int32), ("time_kernels", C.c_int32)]


class Schedule(C.Structure):
    _fields_ = [("size", C.c_uint32), ("n_rungs", C.c_int32), ("absolute", C.c_int32),
                ("tol", C.c_double), ("mu", C.c_double * MAX_RUNGS),
                ("eta_x", C.c_double * MAX_RUNGS), ("eta_k", C.c_double * MAX_RUNGS),
                ("decay", C.c_double * MAX_RUNGS), ("budget", C.c_int64 * MAX_RUNGS)]


class Energy(C.Structure):
    _fields_ = [("E_overlap", C.c_double), ("E_growth", C.c_double),
                ("dE_dkappa_overlap", C.c_double), ("dE_dkappa_growth", C.c_double),
                ("max_overlap", C.c_double), ("n_overlap", C.c_int64)]


class Result(C.Structure):
    _fields_ = [("phi", C.c_double), ("kappa", C.c_double),
                ("kappa_before_shrink", C.c_double), ("max_overlap", C.c_double),
                ("energy", C.c_double), ("iterations", C.c_int64), ("rebuilds", C.c_int64),
                ("status", C.c_int32), ("rung", C.c_int32)]


class Optimizer(C.Structure):
    _fields_ = [("size", C.c_uint32), ("rung", C.c_int32), ("t", C.c_int64),
                ("it_rung", C.c_int64), ("iterations", C.c_int64), ("m_kappa", C.c_double),
                ("v_kappa", C.c_double), ("mu", C.c_double), ("eta_x", C.c_double),
                ("eta_k", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("iterations", C.c_int64), ("particle_updates", C.c_int64),
                ("rebuilds", C.c_int64), ("graph_launches", C.c_int64),
                ("nnz", C.c_int64), ("max_degree", C.c_int64), ("iterate_ms", C.c_double),
                ("rebuild_ms", C.c_double), ("shrink_ms", C.c_double), ("kernel_ms", C.c_double),
                ("tail_kernel_ms", C.c_double), ("kernel_launches", C.c_int64),
                ("kernel_nnz", C.c_int64), ("levels", C.c_int64)]


_lib = None

vp = C.c_void_p
dp = C.POINTER(C.c_double)
i32p = C.POINTER(C.c_int32)
i64p = C.POINTER(C.c_int64)

# name -> (restype, argtypes); mirrors include/rcp.h
SIGNATURES = {
    "rcp_version": (C.c_int, []),
    "rcp_last_error": (C.c_char_p, []),
    "rcp_params_default": (None, [C.POINTER(Params)]),
    "rcp_tuning_default": (None, [C.POINTER(Tuning)]),
    "rcp_schedule_default": (C.c_int, [C.c_int64, C.c_int, C.c_double, C.c_int, C.c_int,
                                       C.c_int64, C.POINTER(Schedule)]),
    "rcp_census_init": (C.c_int, [C.c_int, C.c_int, i64p, C.POINTER(dp), dp, dp,
                                  C.POINTER(C.c_uint64), C.c_int, C.POINTER(Params), vp,
                                  C.POINTER(vp)]),
    "rcp_pack_init": (C.c_int, [C.c_int, dp, C.c_int64, dp, C.c_double, C.c_uint64, C.c_int,
                                C.POINTER(Params), vp, C.POINTER(vp)]),
    "rcp_set_tuning": (C.c_int, [vp, C.POINTER(Tuning)]),
    "rcp_set_skin": (C.c_int, [vp, C.c_double, C.c_double]),
    "rcp_set_state": (C.c_int, [vp, C.c_int, vp, C.c_double, C.c_int]),
    "rcp_get_state": (C.c_int, [vp, C.c_int, dp, dp, dp]),
    "rcp_get_optimizer": (C.c_int, [vp, C.c_int, dp, dp, C.POINTER(Optimizer)]),
    "rcp_set_optimizer": (C.c_int, [vp, C.c_int, dp, dp, C.POINTER(Optimizer)]),
    "rcp_place_device": (C.c_int, [vp, C.c_int, C.c_uint64, C.c_int64, i64p]),
    "rcp_neighbor_build": (C.c_int, [vp, C.c_int, i64p]),
    "rcp_get_pairs": (C.c_int, [vp, C.c_int, i32p, i32p, C.c_int64, i64p]),
    "rcp_energy_grad": (C.c_int, [vp, C.c_int, C.c_double, C.POINTER(Energy), dp]),
    "rcp_adam_step": (C.c_int, [vp, C.c_double, C.c_double, C.c_double, C.c_int64]),
    "rcp_inflate_run": (C.c_int, [vp, C.POINTER(Schedule), C.c_int, C.c_int64,
                                  C.POINTER(Result)]),
    "rcp_census_run": (C.c_int, [vp, C.POINTER(Schedule), C.c_int, C.c_int64,
                                 C.POINTER(Result)]),
    "rcp_run_start": (C.c_int, [vp, C.POINTER(Schedule), C.c_int]),
    "rcp_run_continue": (C.c_int, [vp, C.c_int64, i32p]),
    "rcp_run_prepare": (C.c_int, [vp]),
    "rcp_set_frozen": (C.c_int, [vp, C.c_int, C.c_void_p]),
    "rcp_set_boundary": (C.c_int, [vp, C.c_int, C.c_uint32, C.c_uint32]),
    "rcp_seat_device": (C.c_int, [vp, C.c_int, C.c_double, C.c_uint64, C.c_int64]),
    "rcp_run_result": (C.c_int, [vp, C.c_int, C.POINTER(Result)]),
    "rcp_shrink": (C.c_int, [vp, C.c_int, dp, dp]),
    "rcp_energy_dev": (C.c_int, [vp, vp, C.c_double, C.c_double, vp, vp]),
    "rcp_adjoint_dev": (C.c_int, [vp, vp, C.c_double, C.c_double, vp, vp, vp]),
    "rcp_energy_dev_static": (C.c_int, [vp, vp, C.c_double, C.c_double, vp, vp]),
    "rcp_time_iterations": (C.c_int, [vp, C.c_int64, dp, dp, i64p]),
    "rcp_get_stats": (C.c_int, [vp, C.POINTER(Stats)]),
    "rcp_reset_stats": (C.c_int, [vp]),
    "rcp_num_packings": (C.c_int, [vp]),
    "rcp_num_particles": (C.c_int64, [vp, C.c_int]),
    "rcp_destroy": (None, [vp]),
}


def lib():
    """Load librcp.so; raises if it is missing (build it with build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("librcp.so is not built (%s); run "
                              "paper_2608_12235_amd.build.build()" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(rc):
    if rc != RCP_OK:
        raise RcpError(rc, lib().rcp_last_error().decode())
    return rc
