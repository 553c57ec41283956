"""The C ABI library loads and exports every entry point that include/fmap.h
declares; host-side validation rejects bad problems before touching a GPU."""
import ctypes as C
import os
import re

import pytest

from paper_2005_08661_amd import fmap

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fmap.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fm_[a-z_]+)\s*\(", text)))


def test_header_declares_the_binding_entry_points():
    assert declared_functions() == sorted(fmap.EXPORTED)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(fmap.LIBPATH):
        pytest.skip("libfmap.so not built")
    lib = C.CDLL(fmap.LIBPATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_status_strings_and_host_validation():
    if not os.path.exists(fmap.LIBPATH):
        pytest.skip("libfmap.so not built")
    L = fmap.lib()
    assert L.fm_status_string(0) == b"ok"
    assert L.fm_status_string(5) == b"IC(0) pivot not positive"
    h = C.c_void_p()
    bad = [
        fmap.make_params((0, 4, 4), 1, [0, 1e-3], 0.1),           # empty grid
        fmap.make_params((4, 4, 4), 1, [0.0], 0.1),               # one echo
        fmap.make_params((4, 4, 4), 1, [0, 1e-3], -1.0),          # negative beta
        fmap.make_params((4, 4, 4), 1, [0, 1e-3], 0.1, nmls=0),   # no line search
        fmap.make_params((4, 4, 4), 1, [1e-3, 1e-3], 0.1),        # t_2 == t_1
        fmap.make_params((4, 4, 4), 0, [0, 1e-3], 0.1),           # no coils
        fmap.make_params((4, 4, 4), 1, [0, 1e-3], 0.1, precision=7),
        fmap.make_params((4, 4, 4), 1, [0, 1e-3], 0.1, model=fmap.WATERFAT, fat_hz=[], fat_amp=[]),
    ]
    expect = [2, 2, 1, 1, 1, 2, 1, 1]
    for p, e in zip(bad, expect):
        st = L.fm_plan_create(C.byref(p), C.byref(h))
        assert st == e, (st, e, L.fm_last_error())
        assert not h.value
        assert len(L.fm_last_error()) > 0
    assert L.fm_plan_create(None, C.byref(h)) == 1
    assert L.fm_plan_destroy(None) == 0


def test_size_and_batch_validation_before_any_device_work():
    """Index bound (2^31 padded voxels per plan) and batch compatibility are checked on the host."""
    if not os.path.exists(fmap.LIBPATH):
        pytest.skip("libfmap.so not built")
    L = fmap.lib()
    h = C.c_void_p()
    big = fmap.make_params((2048, 1024, 1024), 1, [0, 1e-3], 0.1)
    assert L.fm_plan_create(C.byref(big), C.byref(h)) == 2 and not h.value
    huge = fmap.make_params((1 << 12, 1 << 12, 1 << 12), 1, [0, 1e-3], 0.1)
    assert L.fm_plan_create(C.byref(huge), C.byref(h)) == 2 and not h.value

    def batch_status(prms):
        arr = (fmap.Params * len(prms))(*prms)
        b = C.c_void_p()
        st = L.fm_batch_create(C.c_int32(len(prms)), C.cast(arr, C.c_void_p), C.byref(b))
        assert not b.value
        return st

    a = fmap.make_params((8, 8, 8), 1, [0, 1e-3, 2e-3], 0.1, ordering=fmap.REDBLACK)
    natural = fmap.make_params((8, 8, 8), 1, [0, 1e-3, 2e-3], 0.1, ordering=fmap.NATURAL)
    other_te = fmap.make_params((8, 8, 8), 1, [0, 1e-3, 2.5e-3], 0.1, ordering=fmap.REDBLACK)
    wf = fmap.make_params((8, 8, 8), 1, [0, 1e-3, 2e-3], 0.1, ordering=fmap.REDBLACK, model=fmap.WATERFAT,
                          fat_hz=[-434.0], fat_amp=[1.0])
    assert batch_status([a, natural]) == 1
    assert batch_status([a, other_te]) == 1
    assert batch_status([a, wf]) == 1
    assert L.fm_batch_create(C.c_int32(0), None, C.byref(h)) == 1
    assert L.fm_batch_destroy(None) == 0


def header_enums():
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    vals = {}
    for body in re.findall(r"enum\s*(?:\w+\s*)?\{([^}]*)\}", text):
        for name, val in re.findall(r"\b(FM_[A-Z0-9_]+)\s*=\s*(-?\d+)", body):
            vals[name] = int(val)
    return vals


def test_binding_constants_match_the_header():
    e = header_enums()
    pairs = {"FM_ORDER_NATURAL": fmap.NATURAL, "FM_ORDER_REDBLACK": fmap.REDBLACK, "FM_ORDER_COLOR3": fmap.COLOR3,
             "FM_ORDER_BLOCKRB": fmap.BLOCKRB,
             "FM_PREC_F64": fmap.F64, "FM_PREC_MIX": fmap.MIX, "FM_FIELDMAP": fmap.FIELDMAP,
             "FM_WATERFAT": fmap.WATERFAT, "FM_SCHED_AUTO": fmap.SCHED_AUTO, "FM_SCHED_STREAM": fmap.SCHED_STREAM,
             "FM_SCHED_RESIDENT": fmap.SCHED_RESIDENT}
    for name, val in pairs.items():
        assert e[name] == val, name


def test_three_colour_order_validation_on_the_host():
    """IC(0) of the second-order C needs the three-colour order, which is built for nothing else;
    both are refused before any device work."""
    if not os.path.exists(fmap.LIBPATH):
        pytest.skip("libfmap.so not built")
    L = fmap.lib()
    h = C.c_void_p()
    te = [0, 1e-3, 2e-3]
    refused = [
        fmap.make_params((8, 8, 8), 1, te, 0.1, ordering=fmap.NATURAL, precond=fmap.IC0, reg_order=2),
        fmap.make_params((8, 8, 8), 1, te, 0.1, ordering=fmap.REDBLACK, precond=fmap.IC0, reg_order=2),
        fmap.make_params((8, 8, 8), 1, te, 0.1, ordering=fmap.COLOR3, precond=fmap.IC0, reg_order=1),
        fmap.make_params((8, 8, 8), 1, te, 0.1, ordering=fmap.COLOR3, precond=fmap.DIAG, reg_order=2),
        fmap.make_params((8, 8, 8), 1, te, 0.1, ordering=3, precond=fmap.IC0, reg_order=2),
    ]
    for p in refused:
        assert L.fm_plan_create(C.byref(p), C.byref(h)) == 1 and not h.value
        assert len(L.fm_last_error()) > 0


def test_ict_pattern_tables_match_the_oracles_symbolic_elimination():
    """The GPU's compile-time IC_t patterns (fm_ict_offsets, host only) equal the level-of-fill patterns
    the oracle derives by symbolic elimination."""
    if not os.path.exists(fmap.LIBPATH):
        pytest.skip("libfmap.so not built")
    import oracle as O
    for level in (0, 1, 2):
        assert fmap.ict_offsets(level) == O.ict_offsets(level)
    with pytest.raises(fmap.FmapError):
        fmap.ict_offsets(3)


def test_ict_parameters_validated_on_the_host():
    if not os.path.exists(fmap.LIBPATH):
        pytest.skip("libfmap.so not built")
    L = fmap.lib()
    h = C.c_void_p()
    bad = [
        fmap.make_params((4, 4, 4), 1, [0, 1e-3], 0.1, precond=fmap.ICT, ordering=fmap.REDBLACK),
        fmap.make_params((4, 4, 4), 1, [0, 1e-3], 0.1, precond=fmap.ICT, ict_level=3),
        fmap.make_params((4, 4, 4), 1, [0, 1e-3], 0.1, precond=fmap.ICT, ict_factor=-1.0),
        fmap.make_params((4, 4, 4), 1, [0, 1e-3], 0.1, precond=fmap.ICT, ict_factor=float("nan")),
        fmap.make_params((4, 4, 4), 1, [0, 1e-3], 0.1, precond=fmap.ICT, reg_order=2),
        fmap.make_params((4, 4, 4), 1, [0, 1e-3], 0.1, precond=4),
    ]
    for p in bad:
        assert L.fm_plan_create(C.byref(p), C.byref(h)) == 1, L.fm_last_error()
        assert not h.value
    arr = (fmap.Params * 2)(*[fmap.make_params((4, 4, 4), 1, [0, 1e-3], 0.1, precond=fmap.ICT)] * 2)
    assert L.fm_batch_create(2, C.cast(arr, C.c_void_p), C.byref(h)) == 1


def test_noalloc_solve_refuses_before_any_device_work():
    """fm_solve_noalloc checks the problem against its fixed workspace on the host: too many voxels or
    iterations give FM_ERR_SHAPE, unsupported modes FM_ERR_ARG, before anything touches a device."""
    if not os.path.exists(fmap.LIBPATH):
        pytest.skip("libfmap.so not built")
    L = fmap.lib()
    dummy = C.c_void_p(16)  # never dereferenced: every case is refused on the host
    cases = [
        (fmap.make_params((128, 128, 64), 1, [0, 1e-3, 2e-3], 0.1, precision=fmap.MIX, ordering=fmap.REDBLACK), 2),
        (fmap.make_params((16, 16, 16), 1, [0, 1e-3, 2e-3], 0.1, niter=5000, ordering=fmap.REDBLACK), 2),
        (fmap.make_params((16, 16, 16), 1, [0, 1e-3, 2e-3], 0.1, ordering=fmap.NATURAL), 1),
        (fmap.make_params((16, 16, 16), 1, [0, 1e-3, 2e-3], 0.1, precond=fmap.ICT), 1),
        (fmap.make_params((16, 16, 16), 1, [0, 1e-3, 2e-3, 3e-3, 4e-3], 0.1, ordering=fmap.REDBLACK), 1),
        (fmap.make_params((16, 16, 16), 1, [1e-3, 2e-3], 0.1, model=fmap.WATERFAT, fat_hz=[-400.0],
                          fat_amp=[1.0], ordering=fmap.REDBLACK), 1),
    ]
    for prm, expect in cases:
        st = L.fm_solve_noalloc(C.byref(prm), dummy, None, dummy, None, dummy, None, None)
        assert st == expect, (st, expect, L.fm_last_error())
    prm = fmap.make_params((16, 16, 16), 1, [0, 1e-3], 0.1, ordering=fmap.REDBLACK)
    assert L.fm_solve_noalloc(C.byref(prm), None, None, dummy, None, dummy, None, None) == 1
