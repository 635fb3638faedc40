"""ctypes loader for libaaqaoa.so (built in-tree by paper_2410_22247_amd/build.py)."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# AAQAOA_LIB names another build of the same sources (the host-sanitizer build of build.py)
LIB_PATH = os.environ.get("AAQAOA_LIB") or os.path.join(HERE, "libaaqaoa.so")

_lib = None


class CProblem(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("num_edges", ctypes.c_int32),
        ("edges", ctypes.POINTER(ctypes.c_int32)),
        ("num_orbits", ctypes.c_int32),
        ("orbit_rep", ctypes.POINTER(ctypes.c_int32)),
        ("orbit_size", ctypes.POINTER(ctypes.c_int32)),
        ("edge_orbit", ctypes.POINTER(ctypes.c_int32)),
        ("edge_weight", ctypes.POINTER(ctypes.c_int32)),
    ]


class CKernelTiming(ctypes.Structure):
    _fields_ = [
        ("name", ctypes.c_char * 32),
        ("launches", ctypes.c_longlong),
        ("total_ms", ctypes.c_double),
        ("bytes", ctypes.c_double),
    ]


class CPlanOpts(ctypes.Structure):
    _fields_ = [
        ("use_graph", ctypes.c_int),
        ("workgroups", ctypes.c_int),
        ("sort_units", ctypes.c_int),
        ("prec", ctypes.c_int),
        ("tile_bits_large", ctypes.c_int),
        ("min_tile_bits_small", ctypes.c_int),
        ("single_launch", ctypes.c_int),
        ("small_streams", ctypes.c_int),
        ("max_small_n", ctypes.c_int),
    ]


EXPORTS = (
    "aaq_validate", "aaq_state_bytes", "aaq_workspace_size", "aaq_energy", "aaq_energy_grad", "aaq_cut_values",
    "aaq_cut_values_layout", "aaq_num_sets", "aaq_plan_default_opts", "aaq_plan_workspace_size", "aaq_plan_create",
    "aaq_plan_execute", "aaq_plan_destroy", "aaq_status_string", "aaq_last_error_message", "aaq_version",
    "aaq_timing_enable", "aaq_timing_read", "aaq_timing_classes", "aaq_set_tile_bits", "aaq_get_tile_bits", "aaq_autotune",
    "aaq_plan_autotune", "aaq_checkpoint_bytes", "aaq_energy_grad_checkpointed", "aaq_lightcone_info",
    "aaq_lightcone_workspace_size", "aaq_lightcone_create", "aaq_lightcone_execute", "aaq_lightcone_destroy",
    "aaq_edge_orbits", "aaq_sample_workspace_size", "aaq_sample", "aaq_resident_workspace_size",
    "aaq_resident_create", "aaq_resident_execute", "aaq_resident_destroy", "aaq_set_half_state",
    "aaq_get_half_state", "aaq_rcc_eta", "aaq_energy_grad_noalloc",
)


def lib():
    """The loaded library.  Raises if it has not been built: there is no fallback."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
                           "or `python paper_2410_22247_amd/build.py`")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER(CProblem)
    vp, sz, i, d = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_double
    dp = ctypes.POINTER(ctypes.c_double)
    szp = ctypes.POINTER(ctypes.c_size_t)
    sig = {
        "aaq_validate": (i, [P, i]),
        "aaq_state_bytes": (i, [P, i, szp]),
        "aaq_workspace_size": (i, [P, i, i, i, i, i, szp]),
        "aaq_energy": (i, [P, i, dp, dp, i, i, i, vp, sz, vp, sz, vp, dp, dp, dp]),
        "aaq_energy_grad": (i, [P, i, dp, dp, i, i, vp, sz, vp, sz, vp, sz, vp, dp, dp, dp, dp]),
        "aaq_energy_grad_noalloc": (i, [P, i, dp, dp, i, i, vp, sz, vp, sz, vp, dp, dp, dp, dp]),
        "aaq_cut_values": (i, [P, i, vp, sz, vp, vp]),
        "aaq_cut_values_layout": (i, [P, i, i, i, i, vp, sz, vp, vp]),
        "aaq_num_sets": (i, [i, i]),
        "aaq_plan_default_opts": (None, [ctypes.POINTER(CPlanOpts)]),
        "aaq_plan_workspace_size": (i, [P, i, i, i, i, ctypes.POINTER(CPlanOpts), szp]),
        "aaq_plan_create": (i, [P, i, i, i, i, ctypes.POINTER(CPlanOpts), vp, sz, vp, ctypes.POINTER(vp)]),
        "aaq_plan_execute": (i, [vp, vp, vp, vp]),
        "aaq_plan_destroy": (None, [vp]),
        "aaq_status_string": (ctypes.c_char_p, [i]),
        "aaq_last_error_message": (ctypes.c_char_p, []),
        "aaq_version": (ctypes.c_char_p, []),
        "aaq_timing_enable": (i, [i]),
        "aaq_timing_classes": (i, [i]),
        "aaq_timing_read": (i, [ctypes.POINTER(CKernelTiming), i, ctypes.POINTER(i), i]),
        "aaq_set_tile_bits": (i, [i, i, i, i]),
        "aaq_checkpoint_bytes": (i, [P, i, i, szp]),
        "aaq_energy_grad_checkpointed": (i, [P, i, dp, dp, i, i, vp, sz, vp, sz, vp, sz, vp, dp, dp, dp, dp]),
        "aaq_get_tile_bits": (i, [i, i, i]),
        "aaq_autotune": (i, [P, i, i, i, i, vp, sz, vp, sz, vp, sz, vp, i, ctypes.POINTER(i), dp]),
        "aaq_plan_autotune": (i, [P, i, i, i, i, ctypes.POINTER(CPlanOpts), vp, sz, vp, vp, vp, i,
                                  ctypes.POINTER(CPlanOpts), dp]),
        "aaq_lightcone_info": (i, [P, i, i, ctypes.POINTER(i), ctypes.POINTER(i), dp]),
        "aaq_lightcone_workspace_size": (i, [P, i, i, i, ctypes.POINTER(CPlanOpts), szp]),
        "aaq_lightcone_create": (i, [P, i, i, i, ctypes.POINTER(CPlanOpts), vp, sz, vp, ctypes.POINTER(vp)]),
        "aaq_lightcone_execute": (i, [vp, vp, vp, vp]),
        "aaq_lightcone_destroy": (None, [vp]),
        "aaq_resident_workspace_size": (i, [P, i, i, i, i, i, szp, szp]),
        "aaq_resident_create": (i, [P, i, i, i, i, i, vp, sz, vp, sz, vp, sz, vp, ctypes.POINTER(vp)]),
        "aaq_resident_execute": (i, [vp, vp, vp, vp]),
        "aaq_resident_destroy": (None, [vp]),
        "aaq_set_half_state": (None, [i]),
        "aaq_get_half_state": (i, []),
        "aaq_sample_workspace_size": (i, [P, i, i, szp]),
        "aaq_sample": (i, [P, i, dp, dp, i, i, vp, vp, sz, vp, sz, vp, vp, vp, dp, dp]),
        "aaq_edge_orbits": (i, [i, i, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
        "aaq_rcc_eta": (i, [i, i, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), i,
                            ctypes.POINTER(ctypes.c_int32), i, dp, dp, ctypes.POINTER(ctypes.c_uint8)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return _lib
