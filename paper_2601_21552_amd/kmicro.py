"""Binding of the gfx950 microbenchmarks (``include/kmicro.h``): measured
int32 VALU, LDS and HBM peaks that the kernels' roofline fractions are
reported against beside the vendor figures."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkmicro.so")


class Peaks(C.Structure):
    _fields_ = [("valu_int32_tops", C.c_double), ("lds_tbs", C.c_double), ("hbm_gbs", C.c_double),
                ("valu_ms", C.c_double), ("lds_ms", C.c_double), ("hbm_ms", C.c_double),
                ("cus", C.c_uint32), ("clock_mhz", C.c_uint32)]


def measure(mib: int = 1024) -> dict:
    """Run the microbenchmarks on the current device with a buffer of `mib`
    MiB (allocated by torch); a dict of the figures."""
    import torch
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2601_21552_amd.build`")
    lib = C.CDLL(LIB_PATH)
    lib.kmicro_run.restype = C.c_int
    lib.kmicro_run.argtypes = [C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(Peaks)]
    buf = torch.ones(mib << 18, dtype=torch.float32, device="cuda")
    p = Peaks()
    st = torch.cuda.current_stream().cuda_stream
    if lib.kmicro_run(C.c_void_p(buf.data_ptr()), buf.numel() * 4, C.c_void_p(st), C.byref(p)) != 0:
        raise RuntimeError("kmicro_run failed")
    del buf
    return {"valu_int32_tops": round(p.valu_int32_tops, 3), "lds_tbs": round(p.lds_tbs, 3),
            "hbm_gbs": round(p.hbm_gbs, 1), "cus": p.cus, "clock_mhz": p.clock_mhz,
            "kernel_ms": {"valu": round(p.valu_ms, 4), "lds": round(p.lds_ms, 4), "hbm": round(p.hbm_ms, 4)}}
