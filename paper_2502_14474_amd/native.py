"""ctypes binding of libmdp.so (the C ABI declared in include/mdp.h).

Argument marshalling only: every step of the solver runs in the HIP library.
Loading fails loudly when the library has not been built; there is no fallback.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmdp.so")

MDP_OK, MDP_W_MAXITER = 0, 1
MDP_E_INVAL, MDP_E_NOMEM, MDP_E_DEVICE, MDP_E_NUMERIC, MDP_E_STATE, MDP_E_NOTSUP = -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "MDP_OK", 1: "MDP_W_MAXITER", -1: "MDP_E_INVAL", -2: "MDP_E_NOMEM",
                -3: "MDP_E_DEVICE", -4: "MDP_E_NUMERIC", -5: "MDP_E_STATE", -6: "MDP_E_NOTSUP"}
MDP_FP64, MDP_MIXED_FP32, MDP_MIXED_FP16 = 0, 1, 2
MDP_INNER_GMRES, MDP_INNER_RICHARDSON, MDP_INNER_BICGSTAB, MDP_INNER_TFQMR = 0, 1, 2, 3
MDP_BUILD_FP32, MDP_BUILD_FP16 = 1, 2
MDP_MINIMIZE_COST, MDP_MAXIMIZE_REWARD = 0, 1
MDP_VALIDATE_NONE, MDP_VALIDATE_HOST, MDP_VALIDATE_DEVICE = 0, 1, 2
MDP_LAUNCH_AUTO, MDP_LAUNCH_GRAPHS, MDP_LAUNCH_DIRECT = 0, 1, 2


class CreateOpts(C.Structure):
    _fields_ = [("struct_size", C.c_size_t), ("stream", C.c_void_p), ("device", C.c_int32),
                ("validate", C.c_int32), ("low_precision", C.c_int32),
                ("lanes_per_row", C.c_int32), ("col_blocks", C.c_int32), ("objective", C.c_int32)]


class EvalOpts(C.Structure):
    _fields_ = [("struct_size", C.c_size_t), ("inner", C.c_int32), ("restart", C.c_int32),
                ("precision", C.c_int32), ("sync_every", C.c_int32), ("rtol", C.c_double),
                ("max_iter", C.c_int64), ("precond_degree", C.c_int32), ("gs_passes", C.c_int32),
                ("policy_copy", C.c_int32)]


class SolveOpts(C.Structure):
    _fields_ = [("struct_size", C.c_size_t), ("inner", C.c_int32), ("restart", C.c_int32),
                ("precision", C.c_int32), ("sync_every", C.c_int32), ("alpha", C.c_double),
                ("atol", C.c_double), ("rtol_cert", C.c_double), ("max_outer", C.c_int64),
                ("max_inner", C.c_int64), ("launch", C.c_int32), ("precond_degree", C.c_int32),
                ("gs_passes", C.c_int32), ("policy_copy", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("struct_size", C.c_size_t), ("outer_iters", C.c_int64),
                ("inner_iters", C.c_int64), ("bellman_sweeps", C.c_int64),
                ("policy_applies", C.c_int64), ("refinements", C.c_int64),
                ("residual", C.c_double), ("time_ms", C.c_double), ("bytes", C.c_double),
                ("history", C.POINTER(C.c_double)), ("history_cap", C.c_int64),
                ("history_len", C.c_int64), ("orth_loss", C.c_double)]


NUM_KERNEL_KINDS = 7
KERNEL_KINDS = ("bellman", "arnoldi_apply", "arnoldi_update", "policy_apply", "gmres_update_x",
                "reduce", "other")


class KernelProfile(C.Structure):
    _fields_ = [("struct_size", C.c_size_t), ("launches", C.c_int64 * NUM_KERNEL_KINDS),
                ("ms", C.c_double * NUM_KERNEL_KINDS), ("bytes", C.c_double * NUM_KERNEL_KINDS)]


class ServerOpts(C.Structure):
    _fields_ = [("struct_size", C.c_size_t), ("stream", C.c_void_p),
                ("hbm_budget_bytes", C.c_int64), ("device", C.c_int32), ("max_batch", C.c_int32),
                ("admit_threads", C.c_int32), ("retire_threads", C.c_int32),
                ("solve", SolveOpts), ("autotune", C.c_int32), ("split_nnz", C.c_int64),
                ("trace_path", C.c_char_p)]


class RequestStats(C.Structure):
    _fields_ = [("struct_size", C.c_size_t), ("submit_ms", C.c_double), ("admit_ms", C.c_double),
                ("finish_ms", C.c_double), ("outer_iters", C.c_int64), ("inner_iters", C.c_int64),
                ("bellman_sweeps", C.c_int64), ("residual", C.c_double), ("bytes", C.c_double)]


# name -> (restype, argtypes); the exported symbols of include/mdp.h
# int32_t (*)(void* user, int64_t s_begin, int64_t s_end, int32_t k_max, int32_t* col,
#            double* val, int32_t* len, double* cost)
ROWS_FN = C.CFUNCTYPE(C.c_int32, C.c_void_p, C.c_int64, C.c_int64, C.c_int32, C.POINTER(C.c_int32),
                      C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_double))

SIGNATURES = {
    "mdp_default_create_opts": (None, [C.POINTER(CreateOpts)]),
    "mdp_create_from_rows": (C.c_int, [C.c_int64, C.c_int32, C.c_int32, ROWS_FN, C.c_void_p, C.c_double,
                                       C.POINTER(CreateOpts), C.POINTER(C.c_void_p)]),
    "mdp_create_from_device_rows": (C.c_int, [C.c_int64, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                              C.c_double, C.POINTER(CreateOpts), C.POINTER(C.c_void_p)]),
    "mdp_load_kernel": (C.c_int, [C.c_char_p, C.c_char_p, C.POINTER(C.c_void_p)]),
    "mdp_default_eval_opts": (None, [C.POINTER(EvalOpts)]),
    "mdp_default_solve_opts": (None, [C.POINTER(SolveOpts)]),
    "mdp_create": (C.c_int, [C.c_int64, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                             C.c_void_p, C.c_double, C.POINTER(CreateOpts),
                             C.POINTER(C.c_void_p)]),
    "mdp_bellman": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                              C.POINTER(C.c_double)]),
    "mdp_policy_apply": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]),
    "mdp_bellman_noalloc": (C.c_int, [C.c_int64, C.c_int32, C.c_int64, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_void_p, C.c_double, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    "mdp_policy_eval": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.POINTER(EvalOpts), C.POINTER(Stats)]),
    "mdp_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                            C.POINTER(SolveOpts), C.POINTER(Stats)]),
    "mdp_solve_batch": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(C.c_void_p),
                                  C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                  C.POINTER(SolveOpts), C.POINTER(Stats)]),
    "mdp_info": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                           C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_int64)]),
    "mdp_autotune": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "mdp_profile": (C.c_int, [C.c_void_p, C.c_int32]),
    "mdp_profile_sampled": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    "mdp_profile_read": (C.c_int, [C.c_void_p, C.POINTER(KernelProfile)]),
    "mdp_default_server_opts": (None, [C.POINTER(ServerOpts)]),
    "mdp_server_create": (C.c_int, [C.POINTER(ServerOpts), C.POINTER(C.c_void_p)]),
    "mdp_server_submit": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_double, C.POINTER(C.c_int64)]),
    "mdp_server_submit_borrowed": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, C.c_void_p,
                                             C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                             C.POINTER(C.c_int64)]),
    "mdp_server_poll": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(C.c_int32)]),
    "mdp_server_wait": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                  C.POINTER(RequestStats)]),
    "mdp_server_info": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                  C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "mdp_server_destroy": (C.c_int, [C.c_void_p]),
    "mdp_destroy": (C.c_int, [C.c_void_p]),
    "mdp_last_error": (C.c_char_p, []),
    "mdp_version": (C.c_char_p, []),
}

_lib = None


def load(path=LIB_PATH):
    """Load libmdp.so and declare its signatures.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run __graft_entry__.build() "
                           "(python paper_2502_14474_amd/build.py)")
    # PyTorch ships its own HIP runtime under the same soname.  Loading torch
    # first lets libmdp.so bind to that one copy; loading libmdp.so first would
    # put a second HIP runtime into the process, and only one can own the GPU.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class MDPError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status):
    if status < 0:
        raise MDPError(status, load().mdp_last_error().decode())
    return status
