"""The C ABI library loads on a CPU host, exports every symbol include/rg.h
declares, and rejects invalid arguments before touching a device."""
import ctypes

import numpy as np
import pytest

from paper_2106_11594_amd import rg


@pytest.fixture(scope="module")
def L():
    return rg.lib()


def test_every_declared_symbol_is_exported(L):
    names = rg.header_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(rg._SIGS), "binding and header disagree"


def test_status_strings(L):
    for code, text in rg._STATUS.items():
        assert L.rg_status_string(code).decode() == text


def test_invalid_arguments_need_no_device(L):
    h = ctypes.c_void_p()
    assert L.rg_init(ctypes.byref(h), 0, None) == 1
    assert L.rg_init(None, 4, None) == 1
    ms = np.array([4, 0], dtype=np.int32)
    assert L.rg_batch_init(ctypes.byref(h), 2, ms.ctypes.data_as(ctypes.c_void_p), None, None) == 1
    ms = np.array([4, 5], dtype=np.int32)
    rmax = np.array([5, 5], dtype=np.int32)  # r_max > m
    assert L.rg_batch_init(ctypes.byref(h), 2, ms.ctypes.data_as(ctypes.c_void_p),
                           rmax.ctypes.data_as(ctypes.c_void_p), None) == 1
    assert L.rg_batch_init(ctypes.byref(h), 0, ms.ctypes.data_as(ctypes.c_void_p), None, None) == 1
    for f in ("rg_push_rows",):
        assert getattr(L, f)(None, None, None, 3) == 1
    assert L.rg_solution(None, None) == 1
    assert L.rg_reset(None) == 1
    assert L.rg_destroy(None) == 1
    r = ctypes.c_int32()
    assert L.rg_rank(None, ctypes.byref(r)) == 1
    assert L.rg_batch_push(None, None, None, None, None) == 1
    assert L.rg_batch_adjoint(None, None, None, None, None, None, None, None) == 1
    assert L.rg_check(None) == 1
    assert L.rg_batch_status(None, None) == 1
    assert L.rg_batch_check_layout(None, None, None, 0, 0) == 1
    ms = np.array([4, 5], dtype=np.int32)
    assert L.rg_batch_init_ws(ctypes.byref(h), 2, ms.ctypes.data_as(ctypes.c_void_p), None, None, None, 1 << 20) == 1


def test_status_codes_match_the_header():
    """The rg_status values of include/rg.h equal the binding's constants."""
    import os
    import re
    hdr = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "rg.h")).read()
    body = hdr.split("typedef enum {", 1)[1].split("} rg_status;", 1)[0]
    vals = {n: int(v) for n, v in re.findall(r"RG_(\w+)\s*=\s*(\d+)", body)}
    assert vals == {"OK": rg.OK, "E_INVALID": rg.E_INVALID, "E_NOMEM": rg.E_NOMEM, "E_DEVICE": rg.E_DEVICE,
                    "E_RANK_CAPACITY": rg.E_RANK_CAPACITY, "E_NONFINITE": rg.E_NONFINITE, "E_STATE": rg.E_STATE,
                    "E_UNSUPPORTED": rg.E_UNSUPPORTED}


def test_default_options(L):
    o = rg.Options()
    o.dtype, o.r_max, o.eps, o.flags = 7, 7, 7.0, 7
    L.rg_default_options(ctypes.byref(o))
    assert (o.dtype, o.r_max, o.eps, o.stream, o.flags) == (rg.RG_F32, 0, -1.0, None, 0)


def test_workspace_bytes_layout():
    """C, Ct (r_max x ldm) and P^-1 (r_max^2) per stream plus w, meta, order."""
    b32 = rg.workspace_bytes([64], [16], "f32")
    b64 = rg.workspace_bytes([64], [16], "f64")
    state32 = (2 * 16 * 64 + 16 * 16) * 4
    assert b32 >= state32 and b64 >= 2 * state32
    assert rg.workspace_bytes([64], None) > rg.workspace_bytes([64], [16])
    assert rg.workspace_bytes([0]) == 0


def test_option_and_flag_bits_match_the_header():
    """Every RG_OPT_* / RG_FLAG_* value in include/rg.h equals the binding's."""
    import os
    import re
    hdr = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "rg.h")).read()
    vals = {n: int(v, 16) for n, v in re.findall(r"#define (RG_(?:OPT|FLAG)_\w+)\s+(0x[0-9a-fA-F]+)u", hdr)}
    assert len(vals) >= 10
    for n, v in vals.items():
        assert getattr(rg, n[3:]) == v, n


def test_both_variant_bits_are_rejected_before_the_device(L):
    o = rg.Options()
    L.rg_default_options(ctypes.byref(o))
    o.flags = rg.OPT_ORTHOGONAL | rg.OPT_ORTHONORMAL
    h = ctypes.c_void_p()
    assert L.rg_init(ctypes.byref(h), 8, ctypes.byref(o)) == 1


def test_pinv_track_rejects_invalid_arguments_before_the_device(L):
    f = L.rg_pinv_track
    nb = L.rg_pinv_track_workspace_bytes
    assert nb(2, 10, 6, 3) == 8 * 2 * (2 * 3 * 6 + 3 * 3 + 10 * 3 + 10)
    assert nb(0, 10, 6, 3) == 0 and nb(1, 10, 6, 7) == 0 and nb(1, -1, 6, 3) == 0
    dummy = ctypes.c_void_p(16)
    args = lambda B, n, m, r, eps, work, wb: (dummy, dummy, B, n, m, r, eps, dummy, dummy, dummy, dummy,
                                               work, wb, None)
    big = 1 << 30
    assert f(*args(0, 10, 6, 3, -1.0, dummy, big)) == 1          # no problems
    assert f(*args(1, 10, 6, 7, -1.0, dummy, big)) == 1          # r_max > m
    assert f(*args(1, 10, 6, 3, float("nan"), dummy, big)) == 1  # NaN threshold
    assert f(*args(1, 10, 6, 3, -1.0, None, big)) == 1           # no workspace
    assert f(*args(1, 10, 6, 3, -1.0, dummy, 8)) == 1            # workspace too small
    assert f(None, None, 1, 10, 6, 3, -1.0, None, dummy, dummy, dummy, dummy, big, None) == 1
    assert f(*args(1, 10, 30000, 3, -1.0, dummy, big)) == rg.E_UNSUPPORTED  # LDS beyond 160 KiB
