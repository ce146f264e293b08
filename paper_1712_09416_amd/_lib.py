"""ctypes declarations of libtpcca.so (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtpcca.so")

TPC_OK, TPC_EINVAL, TPC_ENOMEM, TPC_EOVERFLOW, TPC_EDEVICE, TPC_ESTATE, TPC_EBUSY = 0, -1, -2, -3, -4, -5, -6
TPC_HOST, TPC_DEVICE = 1, 2

ERROR_NAMES = {0: "TPC_OK", -1: "TPC_EINVAL", -2: "TPC_ENOMEM", -3: "TPC_EOVERFLOW",
               -4: "TPC_EDEVICE", -5: "TPC_ESTATE", -6: "TPC_EBUSY"}

EXPORTS = ("tpc_params_default", "tpc_workspace_bytes", "tpc_init_geometry", "tpc_load_clusters",
           "tpc_load_batch", "tpc_track_sector", "tpc_track_event", "tpc_track_events",
           "tpc_submit", "tpc_track_event_streams", "tpc_track_event_noalloc", "tpc_get_tracks",
           "tpc_get_slot_tracks",
           "tpc_device_results", "tpc_get_links", "tpc_kf_step_f32", "tpc_graph_capture",
           "tpc_graph_launch", "tpc_poll", "tpc_set_profiling", "tpc_get_profile",
           "tpc_merge_params_default", "tpc_merge", "tpc_get_merged", "tpc_get_merge_links",
           "tpc_calib_accumulate", "tpc_calib_fit", "tpc_calib_correct_z",
           "tpc_last_error", "tpc_destroy")
STAGES = ("grid", "neighbours", "clean_starts", "tracklets", "weights_select", "refit", "output")
COUNTERS = ("tracklets", "row_visits", "window_hits", "tracks_refitted", "clusters", "sorted_hits",
            "tracklet_hits", "update_tries", "tracks", "track_hits")


class Geometry(ctypes.Structure):
    _fields_ = [("n_sectors", ctypes.c_int32), ("n_rows", ctypes.c_int32),
                ("row_x", ctypes.c_float * 160), ("bz_tesla", ctypes.c_float),
                ("tan_half_angle", ctypes.c_float), ("z_max", ctypes.c_float),
                ("sigma_y0", ctypes.c_float), ("sigma_y1", ctypes.c_float),
                ("sigma_z0", ctypes.c_float), ("sigma_z1", ctypes.c_float)]


class Params(ctypes.Structure):
    _fields_ = [("nf_window", ctypes.c_float), ("nf_mmax", ctypes.c_float),
                ("chi2_max", ctypes.c_float), ("k_win", ctypes.c_float),
                ("w_max", ctypes.c_float), ("s_max", ctypes.c_float),
                ("c_s0", ctypes.c_float), ("c_t0", ctypes.c_float), ("c_q0", ctypes.c_float),
                ("m_edge", ctypes.c_float), ("m_z", ctypes.c_float),
                ("n_gap", ctypes.c_int32), ("n_min_tracklet", ctypes.c_int32),
                ("n_min_track", ctypes.c_int32), ("bin_target", ctypes.c_float),
                ("bin_min_edge", ctypes.c_float), ("max_slots", ctypes.c_int32),
                ("max_events", ctypes.c_int32), ("max_clusters", ctypes.c_int64),
                ("x0_cm", ctypes.c_float), ("ms_mass", ctypes.c_float),
                ("n_min_chain", ctypes.c_int32), ("tl_block", ctypes.c_int32),
                ("win_batch", ctypes.c_int32), ("row_batch", ctypes.c_int32)]


class MergeParams(ctypes.Structure):
    _fields_ = [("chi2_max", ctypes.c_float), ("row_gap", ctypes.c_int32),
                ("step_max", ctypes.c_float), ("passes", ctypes.c_int32),
                ("s_max", ctypes.c_float)]


TRACK_DTYPE = np.dtype([("event", "<i4"), ("sector", "<i4"), ("n_hits", "<i4"),
                        ("row_in", "<i4"), ("row_out", "<i4"), ("ndf", "<i4"),
                        ("hit_off", "<i8"), ("inner_id", "<i4"), ("start_id", "<i4"),
                        ("x_ref", "<f8"), ("par", "<f8", (5,)), ("cov", "<f8", (15,)),
                        ("chi2", "<f8")], align=True)
assert TRACK_DTYPE.itemsize == 216

_lib = None


class NativeMissing(RuntimeError):
    pass


def load() -> ctypes.CDLL:
    """Load the HIP library; raises if it was not built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise NativeMissing(f"{LIB_PATH} not built: run `python -m paper_1712_09416_amd.build` "
                            "or __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    P, I, I64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
    L.tpc_params_default.argtypes = [ctypes.POINTER(Params)]
    L.tpc_workspace_bytes.restype = ctypes.c_size_t
    L.tpc_workspace_bytes.argtypes = [ctypes.POINTER(Params)]
    L.tpc_init_geometry.argtypes = [ctypes.POINTER(P), ctypes.POINTER(Geometry),
                                    ctypes.POINTER(Params), P, ctypes.c_size_t, P]
    L.tpc_load_clusters.argtypes = [P, I, P, P, P, P, P, I64, I]
    L.tpc_load_batch.argtypes = [P, I, I, P, P, P, P, P, P, I]
    L.tpc_track_sector.argtypes = [P, I, I]
    L.tpc_track_event.argtypes = [P, I]
    L.tpc_track_events.argtypes = [P, P, I]
    L.tpc_submit.argtypes = [P, I]
    L.tpc_track_event_streams.argtypes = [P, I, I]
    L.tpc_track_event_noalloc.argtypes = [ctypes.POINTER(Geometry), ctypes.POINTER(Params), P, P, P,
                                          P, I64, P, I64, P, I64, P, P]
    L.tpc_get_tracks.argtypes = [P, I, I, P, I64, P, I64, P, P]
    L.tpc_get_slot_tracks.argtypes = [P, I, P, I64, P, I64, P, P, P, P]
    L.tpc_device_results.argtypes = [P, I, P, P, P, P, P]
    L.tpc_get_links.argtypes = [P, I, I, P, P, P, P]
    L.tpc_kf_step_f32.argtypes = [P, P, P, P, P, I64]
    L.tpc_graph_capture.argtypes = [P, I]
    L.tpc_graph_launch.argtypes = [P, I]
    L.tpc_poll.argtypes = [P, I]
    L.tpc_set_profiling.argtypes = [P, I]
    L.tpc_get_profile.argtypes = [P, P, P]
    L.tpc_merge_params_default.argtypes = [ctypes.POINTER(MergeParams)]
    L.tpc_merge.argtypes = [P, I, ctypes.POINTER(MergeParams)]
    L.tpc_get_merged.argtypes = [P, I, I, P, I64, P, I64, P, P, P]
    L.tpc_get_merge_links.argtypes = [P, I, I, P, P, P, P]
    F, D = ctypes.c_float, ctypes.c_double
    L.tpc_calib_accumulate.argtypes = [P, I, P, I, F, F]
    L.tpc_calib_fit.argtypes = [P, I, F, F, F, D, P, P]
    L.tpc_calib_correct_z.argtypes = [P, P, P, I64, D]
    L.tpc_last_error.restype = ctypes.c_char_p
    L.tpc_last_error.argtypes = [P]
    L.tpc_destroy.argtypes = [P]
    _lib = L
    return L


class TpcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


def check(rc: int, ctx=None):
    if rc != TPC_OK:
        msg = load().tpc_last_error(ctx)
        raise TpcError(rc, msg.decode() if msg else "")
    return rc
