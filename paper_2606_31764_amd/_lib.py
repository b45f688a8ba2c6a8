"""ctypes view of the C ABI in include/nsplat.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnsplat.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "nsplat.h")

OK, EINVAL, ECAPACITY, EHIP = 0, 1, 2, 3
CLOSED, FILLED, ANISO = 1, 2, 4
MAX_DEGREE = 5
ABI_VERSION = 7  # NSPLAT_ABI_VERSION of include/nsplat.h
CNT_GAUSS, CNT_PAIRS, CNT_STATUS, CNT_GAUSS_REQ, CNT_PAIRS_REQ, CNT_BOUND_REQ, CNT_BOUND = range(7)
NUM_COUNTERS = 16
STATUS_GAUSS_CAP, STATUS_PAIR_CAP, STATUS_BOUND_CAP, STATUS_DATA, STATUS_VALUE = 1, 2, 4, 8, 16
PLAN_STRIDE = 9
PLAN_FLAGS = 8
PLAN_NEAR_INT, PLAN_INVALID = 1, 2

vp = ctypes.c_void_p


class Curves(ctypes.Structure):
    _fields_ = [("n_curves", ctypes.c_int32), ("channels", ctypes.c_int32), ("n_keys", ctypes.c_int32),
                ("n_taus", ctypes.c_int32), ("max_degree", ctypes.c_int32), ("any_flags", ctypes.c_int32),
                ("all_flags", ctypes.c_int32)] + [
                    (n, vp) for n in (
                    "scene", "degree", "flags", "key_off", "tau_off", "key_xy", "key_w", "key_s", "tau",
                    "color", "opacity")]


class Scenes(ctypes.Structure):
    _fields_ = [("n_scenes", ctypes.c_int32), ("hw_host", vp), ("hw", vp), ("bg", vp)]


class Params(ctypes.Structure):
    _fields_ = [(n, ctypes.c_float) for n in ("delta_c", "delta_b", "rho", "eta", "gamma", "nl_factor", "fill_pad",
                                               "h", "k_sigma", "alpha_max", "eps_T", "delta_a")] + [
        ("kappa", ctypes.c_int32), ("tile", ctypes.c_int32), ("batch", ctypes.c_int32), ("chunk", ctypes.c_int32),
        ("h_dev", vp)]


class Caps(ctypes.Structure):
    _fields_ = [("gauss", ctypes.c_int64), ("pairs", ctypes.c_int64), ("boundary", ctypes.c_int64)]


class Buffers(ctypes.Structure):
    _fields_ = [("plan", vp), ("gauss", vp), ("ranges", vp), ("idx", vp), ("counters", vp), ("ws", vp),
                ("ws_bytes", ctypes.c_size_t), ("caps", Caps)]


class Grads(ctypes.Structure):
    _fields_ = [(n, vp) for n in ("key_xy", "key_w", "key_s", "tau", "color", "opacity")]


class Reg(ctypes.Structure):
    _fields_ = [("bbox_weight", ctypes.c_float), ("bbox_kind", ctypes.c_int32), ("bbox", vp),
                ("deriv_weight", ctypes.c_float), ("deriv_order", ctypes.c_int32), ("loss", vp)]


class Values(ctypes.Structure):
    _fields_ = [("n_curves", ctypes.c_int32), ("channels", ctypes.c_int32), ("n_keys", ctypes.c_int32),
                ("n_taus", ctypes.c_int32)] + [(n, vp) for n in ("key_xy", "key_w", "key_s", "tau", "color",
                                                                   "opacity")]


class Adam(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float * 6), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("final_ratio", ctypes.c_float), ("total_steps", ctypes.c_int32),
                ("w_min", ctypes.c_float), ("w_max", ctypes.c_float), ("tau_min", ctypes.c_float),
                ("tau_max", ctypes.c_float)]


_SIGS = {
    "nsplat_abi_version": (ctypes.c_int, []),
    "nsplat_create": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.c_int]),
    "nsplat_destroy": (ctypes.c_int, [vp]),
    "nsplat_last_error": (ctypes.c_char_p, [vp]),
    "nsplat_num_tiles": (ctypes.c_int64, [vp, ctypes.c_int32]),
    "nsplat_workspace_size": (ctypes.c_size_t, [vp, vp, vp, vp]),
    "nsplat_sample": (ctypes.c_int, [vp, vp, vp, vp, vp, ctypes.c_int, vp]),
    "nsplat_bin": (ctypes.c_int, [vp, vp, vp, vp, vp, vp]),
    "nsplat_forward": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_int, vp]),
    "nsplat_backward": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_int, vp]),
    "nsplat_backward_reg": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_int, vp]),
    "nsplat_adam_step": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, vp, vp]),
    "nsplat_udf_loss": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, ctypes.c_float, vp, vp, vp, vp, vp]),
    "nsplat_udf_loss_noalloc": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, ctypes.c_float, vp, vp, vp, vp, vp]),
    "nsplat_anneal_h": (ctypes.c_int, [vp, vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_float, ctypes.c_float,
                                       ctypes.c_float, ctypes.c_float, vp]),
    "nsplat_l2_grad": (ctypes.c_int, [vp, vp, vp, vp, vp, ctypes.c_int64, vp]),
    "nsplat_read_counters": (ctypes.c_int, [vp, vp, vp, vp]),
    "nsplat_gauss_frame": (ctypes.c_int, [vp, vp, vp, vp, vp, ctypes.c_int64, vp]),
    "nsplat_autotune": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_int, vp, vp, vp, vp]),
}

_lib = None


def header_symbols():
    """Function names declared in include/nsplat.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(nsplat_[a-z0-9_]+)\s*\(", txt)))


def load():
    """Loads the in-tree libnsplat.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        # torch first: it loads the HIP runtime it ships, and the library's
        # libamdhip64.so.7 then binds to that same copy.  Loaded the other way
        # round, torch pulls in a second runtime beside the system one and the
        # two do not see each other's devices.
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libnsplat.so is not built: run `python -c 'import __graft_entry__ as g; g.build()'`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(lib, name)
            f.restype, f.argtypes = res, args
        # the structures below are laid out for this version only
        if lib.nsplat_abi_version() != ABI_VERSION:
            raise RuntimeError("libnsplat.so has ABI version %d, this binding expects %d: rebuild it"
                               % (lib.nsplat_abi_version(), ABI_VERSION))
        _lib = lib
    return _lib


class NSplatError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("nsplat error %d: %s" % (code, msg))
        self.code = code


def check(ctx, rc):
    if rc != OK:
        msg = load().nsplat_last_error(ctx)
        raise NSplatError(rc, msg.decode() if msg else "")
    return rc
