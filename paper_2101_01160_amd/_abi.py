"""ctypes declarations of libmdlg.so (the C ABI in include/mdlg.h).

Loads the in-tree library built by paper_2101_01160_amd/build.py and fails
loudly when it is missing: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libmdlg.so")

MDLG_OK = 0
STATUS_NAMES = {0: "MDLG_OK", -1: "MDLG_EINVAL", -2: "MDLG_ENOMEM", -3: "MDLG_EHIP", -4: "MDLG_ENONFINITE",
                -5: "MDLG_ESKIN", -6: "MDLG_ENOTIMPL", -7: "MDLG_ECAPACITY",
                -8: "MDLG_ERANGE"}

# every symbol declared in include/mdlg.h
EXPORTS = [
    "mdlg_last_error", "mdlg_version", "mdlg_velocity_table",
    "lj_md_init", "lj_md_init_batch", "lj_md_cg_attach", "lj_md_cg_detach", "lj_md_step", "lj_md_step_timed",
    "lj_md_get_state", "lj_md_forces", "lj_md_energy", "lj_md_check", "lj_md_info", "lj_md_save", "lj_md_load", "lj_md_destroy",
    "lj_md_autotune",
    "mdlg_coarse_grain", "mdlg_coarse_grain_noalloc", "mdlg_coarse_grain_series", "mdlg_feq_measured", "mdlg_moments", "mdlg_lambda_from_moments",
    "mdlg_feq_gauss", "mdlg_feq_wsg",
    "mdlg_neq_mdlg", "mdlg_vacf", "mdlg_lambda_vacf", "mdlg_displacement_hist", "mdlg_pdf_bins", "mdlg_pdf_measured", "mdlg_kl_divergence",
    "mdlg_mlp_create", "mdlg_mlp_params", "mdlg_mlp_forward", "mdlg_mlp_gradient", "mdlg_mlp_train_step",
    "mdlg_feq_surrogate", "mdlg_mlp_destroy",
    "mdlg_moment_table_create", "mdlg_moment_table_eval", "mdlg_moment_table_info", "mdlg_moment_table_destroy",
    "mdlg_feq_surrogate_table",
]

MLP_NPARAMS = 145969
HIST_MAX_BINS = 4094
NOALLOC_MAX_N = 1 << 25  # particles of one mdlg_coarse_grain_noalloc call


class LJParams(C.Structure):
    _fields_ = [
        ("n", C.c_int64),
        ("box_l", C.c_double),
        ("dt", C.c_double),
        ("rc", C.c_double),
        ("eps", C.c_double),
        ("energy_shift", C.c_int32),
        ("force_bits", C.c_int32),
        ("skin", C.c_double),
        ("rebuild_every", C.c_int32),
        ("block_size", C.c_int32),
        ("step_kernel", C.c_int32),
        ("gather_batch", C.c_int32),
        ("fuse_steps", C.c_int32),
    ]


class Lattice(C.Structure):
    _fields_ = [("lx", C.c_int32), ("reserved", C.c_int32), ("u", C.c_double * 2)]


class Info(C.Structure):
    _fields_ = [
        ("n_rep", C.c_int32),
        ("rebuild_every", C.c_int32),
        ("n_total", C.c_int64),
        ("steps_done", C.c_int64),
        ("events_done", C.c_int64),
        ("cells_per_side", C.c_int32),
        ("block_size", C.c_int32),
        ("cell_width", C.c_double),
        ("steps_per_launch", C.c_int32),
        ("reserved", C.c_int32),
    ]


_lib = None


class MDLGError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def _init_device_runtime():
    """PyTorch carries its own copy of the HIP runtime.  Its device context is
    brought up before the library (linked to the system HIP runtime) loads:
    loaded the other way round, the library's first HIP call can report that
    no device exists."""
    try:
        import torch
    except ImportError:
        return
    if torch.cuda.is_available():
        torch.cuda.init()
        torch.cuda.current_stream().synchronize()


def lib() -> C.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise ImportError(f"libmdlg.so is not built ({LIBPATH}); run __graft_entry__.build() or "
                          "python paper_2101_01160_amd/build.py")
    _init_device_runtime()
    L = C.CDLL(LIBPATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    P = C.POINTER
    sig = {
        "mdlg_last_error": (C.c_char_p, []),
        "mdlg_version": (C.c_char_p, []),
        "mdlg_velocity_table": (i32, [vp]),
        "lj_md_init": (i32, [P(vp), P(LJParams), vp, vp, vp]),
        "lj_md_init_batch": (i32, [P(vp), i32, P(LJParams), vp, vp, vp]),
        "lj_md_cg_attach": (i32, [vp, i32, P(Lattice), vp, vp, vp, vp]),
        "lj_md_cg_detach": (i32, [vp]),
        "lj_md_step": (i32, [vp, i64, vp]),
        "lj_md_step_timed": (i32, [vp, i64, i32, vp, vp, vp]),
        "lj_md_get_state": (i32, [vp, vp, vp, vp, vp]),
        "lj_md_forces": (i32, [vp, vp, vp]),
        "lj_md_energy": (i32, [vp, vp, vp]),
        "lj_md_check": (i32, [vp, vp]),
        "lj_md_info": (i32, [vp, P(Info)]),
        "lj_md_save": (i32, [vp, C.c_char_p, vp]),
        "lj_md_load": (i32, [P(vp), C.c_char_p, vp]),
        "lj_md_destroy": (None, [vp]),
        "lj_md_autotune": (i32, [i32, P(LJParams), vp, vp, i32, P(Lattice), i32, P(LJParams), P(dbl), vp]),
        "mdlg_coarse_grain": (i32, [P(Lattice), dbl, i64, vp, vp, i64, vp, vp, i64, vp, vp, vp, vp, vp]),
        "mdlg_coarse_grain_noalloc": (i32, [P(Lattice), dbl, i64, vp, vp, i64, vp, vp, i64, vp, vp, vp, vp, vp]),
        "mdlg_coarse_grain_series": (i32, [i32, vp, vp, vp, i32, vp, vp, i32, vp, i32, vp, vp, vp, vp, vp]),
        "mdlg_feq_measured": (i32, [vp, i64, i64, i32, vp, P(dbl)]),
        "mdlg_moments": (i32, [vp, dbl, P(dbl), P(dbl), P(dbl)]),
        "mdlg_lambda_from_moments": (i32, [dbl, dbl, i32, P(dbl), P(dbl)]),
        "mdlg_feq_gauss": (i32, [dbl, vp, vp]),
        "mdlg_feq_wsg": (i32, [dbl, dbl, vp, vp]),
        "mdlg_vacf": (i32, [i32, vp, i32, vp, i32, vp, vp, vp]),
        "mdlg_lambda_vacf": (i32, [i32, vp, vp, dbl, dbl, P(dbl), P(dbl)]),
        "mdlg_neq_mdlg": (i32, [i64, dbl, i32, i32, vp, vp, vp, vp, vp, vp]),
        "mdlg_displacement_hist": (i32, [i32, vp, vp, i32, vp, vp, i32, vp, vp, i32, vp, vp]),
        "mdlg_pdf_bins": (i32, [dbl, dbl, dbl, dbl, i32, vp, vp]),
        "mdlg_pdf_measured": (i32, [vp, i32, i32, vp]),
        "mdlg_kl_divergence": (i32, [vp, vp, i32, vp, P(dbl)]),
        "mdlg_mlp_create": (i32, [P(vp), vp, i32, vp]),
        "mdlg_mlp_params": (i32, [vp, vp, vp]),
        "mdlg_mlp_forward": (i32, [vp, vp, i32, vp, vp]),
        "mdlg_mlp_gradient": (i32, [vp, vp, vp, i32, vp, vp, vp]),
        "mdlg_mlp_train_step": (i32, [vp, vp, vp, i32, C.c_float, vp, vp]),
        "mdlg_feq_surrogate": (i32, [vp, vp, dbl, dbl, dbl, vp, P(i32), P(dbl), vp]),
        "mdlg_mlp_destroy": (None, [vp]),
        "mdlg_moment_table_create": (i32, [P(vp), vp, i64, vp, vp, vp, dbl, i32]),
        "mdlg_moment_table_eval": (i32, [vp, vp, P(dbl), P(dbl), P(dbl)]),
        "mdlg_moment_table_info": (i32, [vp, vp, vp, vp, vp]),
        "mdlg_moment_table_destroy": (None, [vp]),
        "mdlg_feq_surrogate_table": (i32, [vp, vp, vp, dbl, vp, P(i32), P(dbl), P(dbl), P(dbl), vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def check(status: int):
    if status != MDLG_OK:
        msg = lib().mdlg_last_error().decode(errors="replace")
        raise MDLGError(status, msg)
