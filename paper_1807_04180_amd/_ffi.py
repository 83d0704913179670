"""ctypes declarations of the libddm C-ABI (include/ddm.h)."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libddm.so")

DDM_OK, DDM_EINVAL, DDM_ENOMEM, DDM_ESINGULAR, DDM_EHIP, DDM_ESTATE = 0, -1, -2, -3, -4, -5
DDM_ENOCONV, DDM_EDIVERGED = 1, 2
DDM_FP64, DDM_MIXED = 0, 1
DDM_STATIONARY, DDM_FGMRES = 0, 1

STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "ESINGULAR", -4: "EHIP", -5: "ESTATE",
                1: "ENOCONV", 2: "EDIVERGED"}


class DdmProblem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("M", ctypes.c_int * 3), ("h", ctypes.c_double),
                ("n_pml", ctypes.c_int), ("sigma0", ctypes.c_double), ("N", ctypes.c_int * 3),
                ("n_ov", ctypes.c_int), ("precision", ctypes.c_int), ("hbm_budget_bytes", ctypes.c_size_t),
                ("reflection", ctypes.c_double), ("k2_on_host", ctypes.c_int)]


class DdmSolveOpts(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int), ("tol", ctypes.c_double), ("maxiter", ctypes.c_int),
                ("restart", ctypes.c_int), ("K", ctypes.c_int), ("refine_every", ctypes.c_int),
                ("check_every", ctypes.c_int)]


class DdmRhsInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("local_solves", ctypes.c_int), ("relres", ctypes.c_double),
                ("seconds", ctypes.c_double), ("status", ctypes.c_int)]


class DdmProfile(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_long * 4), ("ms", ctypes.c_double * 4), ("bytes", ctypes.c_double * 4)]


KERNEL_CLASSES = ("substitution", "transfer", "assembly", "residual")
SOLVE_VARIANTS = ("perline", "chain", "chain2", "mma")
TRANSFER_FORMS = ("direct", "phi")   # DDM_TRANSFER_DIRECT, DDM_TRANSFER_PHI

_lib = None


class LibraryMissing(ImportError):
    pass


def lib():
    """Load libddm.so (built in-tree by paper_1807_04180_amd.build); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LibraryMissing("libddm.so not found at %s: build it with `python -m paper_1807_04180_amd.build` "
                             "(there is no CPU fallback)" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    H = ctypes.c_void_p
    LP = ctypes.POINTER(ctypes.c_long)
    DP = ctypes.POINTER(ctypes.c_double)
    L.ddm_version.restype = ctypes.c_char_p
    L.ddm_last_error.restype = ctypes.c_char_p
    L.ddm_last_error.argtypes = [H]
    L.ddm_memory_required.argtypes = [ctypes.POINTER(DdmProblem), I, ctypes.POINTER(ctypes.c_size_t)]
    L.ddm_setup.argtypes = [ctypes.POINTER(DdmProblem), P, I, P, ctypes.POINTER(H)]
    L.ddm_factor.argtypes = [H]
    L.ddm_iterate.argtypes = [H, P, P, I, I, DP]
    L.ddm_solve.argtypes = [H, P, P, I, ctypes.POINTER(DdmSolveOpts), ctypes.POINTER(DdmRhsInfo)]
    L.ddm_destroy.argtypes = [H]
    L.ddm_destroy.restype = None
    L.ddm_sizes.argtypes = [H, LP]
    L.ddm_pml_strength.argtypes = [H, DP]
    L.ddm_device_bytes.argtypes = [H, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]
    L.ddm_geometry.argtypes = [H, I, LP]
    L.ddm_apply.argtypes = [H, P, P, I]
    L.ddm_residual.argtypes = [H, P, P, P, I, DP, DP]
    L.ddm_residual_noalloc.argtypes = [H, P, P, P, I, P]
    L.ddm_restrict_core.argtypes = [H, P, P, I]
    L.ddm_local_solve.argtypes = [H, P, P, I]
    L.ddm_transfer.argtypes = [H, P, P, P, P, I]
    L.ddm_assemble.argtypes = [H, P, P, I]
    L.ddm_slot_admit.argtypes = [H, I, P]
    L.ddm_slots_step.argtypes = [H, I]
    L.ddm_slots_poll.argtypes = [H, DP, ctypes.POINTER(ctypes.c_int)]
    L.ddm_slot_retire.argtypes = [H, I, P]
    L.ddm_set_graphs.argtypes = [H, I]
    L.ddm_graph_launches.argtypes = [H]
    L.ddm_graph_launches.restype = ctypes.c_long
    L.ddm_set_factor_layout.argtypes = [H, I]
    L.ddm_set_solve_variant.argtypes = [H, I]
    L.ddm_get_solve_variant.argtypes = [H]
    L.ddm_autotune.argtypes = [H, I, I, DP]
    L.ddm_set_spin_limit.argtypes = [H, I]
    L.ddm_set_chain_tile.argtypes = [H, I]
    L.ddm_time_local_solve.argtypes = [H, I, I, DP]
    L.ddm_set_transfer_form.argtypes = [H, I]
    L.ddm_profile_enable.argtypes = [H, I]
    L.ddm_profile_read.argtypes = [H, ctypes.POINTER(DdmProfile)]
    for name in ("ddm_slot_admit", "ddm_slots_step", "ddm_slots_poll", "ddm_slot_retire", "ddm_set_graphs", "ddm_set_factor_layout", "ddm_set_solve_variant", "ddm_get_solve_variant", "ddm_autotune", "ddm_set_spin_limit", "ddm_set_chain_tile", "ddm_time_local_solve", "ddm_set_transfer_form",
                 "ddm_profile_enable", "ddm_profile_read", "ddm_memory_required", "ddm_setup", "ddm_factor", "ddm_iterate", "ddm_solve", "ddm_sizes",
                 "ddm_geometry", "ddm_apply", "ddm_residual", "ddm_residual_noalloc", "ddm_restrict_core", "ddm_local_solve",
                 "ddm_transfer", "ddm_assemble", "ddm_pml_strength", "ddm_device_bytes"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def header_functions():
    """Names of the functions include/ddm.h declares."""
    import re
    path = os.path.join(os.path.dirname(HERE), "include", "ddm.h")
    with open(path) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ddm_[a-z0-9_]+)\s*\(", text)))
