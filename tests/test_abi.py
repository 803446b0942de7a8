"""CPU checks of the C-ABI boundary: the library loads, exports every symbol
include/mpir.h declares, and its host-side argument validation answers
without touching a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mpir.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mpir_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def M():
    from paper_2311_14616_amd import mpir
    if not os.path.exists(mpir.LIB_PATH):
        pytest.fail("libmpir.so is not built (run __graft_entry__.build())")
    mpir.lib()
    return mpir


def test_every_declared_symbol_is_exported(M):
    names = _declared()
    assert len(names) >= 14
    lib = M.lib()
    missing = [nm for nm in names if not hasattr(lib, nm)]
    assert not missing
    assert set(M.EXPORTS) <= set(names)


def test_status_strings(M):
    for st in (M.OK, M.ERR_SINGULAR, M.ERR_ARG, M.ERR_ALLOC, M.ERR_HIP, M.ERR_NONFINITE,
               M.ERR_RANGE, M.ERR_STATE, M.ERR_DEVICE):
        assert M.status_str(st) and M.status_str(st) != "unknown status"
    assert M.status_str(12345) == "unknown status"


def test_term_defaults_match_paper(M):
    # section "Changing the parameters": Cr = Ce = 1, Rmax = .5, litmax = 10
    t = M.Term()
    M.lib().mpir_term_default(C.byref(t))
    assert (t.Cr, t.Ce, t.Rmax, t.litmax, t.residterm, t.tol_rel) == (1.0, 1.0, 0.5, 10, 1, 0.0)


def test_argument_validation_needs_no_device(M):
    L = M.lib()
    h = C.c_void_p(0)
    info = C.c_int64(7)
    dummy = C.c_void_p(0x1000)
    # n <= 0, lda < n, null pointer, bad precision triples: rejected before any HIP call
    assert L.mpir_factor(0, dummy, 1, M.F64, M.F32, M.F64, None, C.byref(h), C.byref(info)) == M.ERR_ARG
    assert L.mpir_factor(8, dummy, 4, M.F64, M.F32, M.F64, None, C.byref(h), C.byref(info)) == M.ERR_ARG
    assert L.mpir_factor(8, None, 8, M.F64, M.F32, M.F64, None, C.byref(h), C.byref(info)) == M.ERR_ARG
    assert L.mpir_factor(8, dummy, 8, M.F32, M.F64, M.F64, None, C.byref(h), C.byref(info)) == M.ERR_ARG
    assert L.mpir_factor(8, dummy, 8, M.F64, 7, M.F64, None, C.byref(h), C.byref(info)) == M.ERR_ARG
    assert L.mpir_factor(8, dummy, 8, M.BF16, M.BF16, M.F64, None, C.byref(h), C.byref(info)) == M.ERR_ARG
    assert L.mpir_factor(8, dummy, 8, M.F64, M.F32, M.F32, None, C.byref(h), C.byref(info)) == M.ERR_ARG
    assert h.value in (None, 0) and info.value == 0
    assert L.mpir_solve(None, dummy, dummy) == M.ERR_ARG
    assert L.mpir_ir_solve(None, dummy, dummy, None, None) == M.ERR_ARG
    assert L.mpir_gmres_ir_solve(None, dummy, dummy, None, 10, 0.0, None, None) == M.ERR_ARG
    assert L.mpir_bicgstab_ir_solve(None, dummy, dummy, None, 10, 0.0, None, None) == M.ERR_ARG
    assert L.mpir_ir_solve_multi(None, 2, dummy, 8, dummy, 8, None, None) == M.ERR_ARG
    assert L.mpir_refactor(None, dummy, 8, None) == M.ERR_ARG
    assert L.mpir_get_factors(None, dummy, None) == M.ERR_ARG
    assert L.mpir_prof_get(99, None, None, None) == M.ERR_ARG
    assert L.mpir_batch_phase_times(None, 0) == M.ERR_ARG
    L.mpir_destroy(None)


def test_binding_has_no_cpu_fallback():
    # the product path must not reach the oracle or any host solver
    src = open(os.path.join(ROOT, "paper_2311_14616_amd", "mpir.py")).read()
    assert "oracle" not in src.replace("no fallback", "")
    assert "numpy.linalg" not in src and "scipy" not in src and "torch.linalg" not in src


def test_batch_tuning_table_host_logic():
    """The tuning table is host state: defaults, validated replacement and
    reset work without a device."""
    from paper_2311_14616_amd import mpir as M
    d0 = M.batch_get_tuning(M.F64, M.F16).as_dict()
    assert d0["classes"][-1]["nmax"] == 1024 and not d0["from_cache"]
    assert all(c["panel"] in (16, 32) and c["update"] in (0, 1) for c in d0["classes"])
    t = M.batch_get_tuning(M.F64, M.F16)
    t.panel[0], t.update[0] = 16, 1
    M.batch_set_tuning(M.F64, M.F16, t)
    c0 = M.batch_get_tuning(M.F64, M.F16).as_dict()["classes"][0]
    assert (c0["panel"], c0["update"]) == (16, 1)
    # other precision pairs keep their own table
    assert M.batch_get_tuning(M.F64, M.F32).as_dict()["classes"][0]["panel"] == d0["classes"][0]["panel"]
    # panels in pairs (update form 2) need 32-column panels
    t.panel[0], t.update[0] = 32, 2
    M.batch_set_tuning(M.F64, M.F16, t)
    for bad in ({"panel": 8}, {"update": 3}, {"update": -1}, {"panel": 16, "update": 2},
                {"nmax_last": 512}, {"nclass": 0}, {"nclass": 9}):
        u = M.batch_get_tuning(M.F64, M.F16)
        if "panel" in bad:
            u.panel[1] = bad["panel"]
        if "update" in bad:
            u.update[1] = bad["update"]
        if "nmax_last" in bad:
            u.nmax[u.nclass - 1] = bad["nmax_last"]
        if "nclass" in bad:
            u.nclass = bad["nclass"]
        with pytest.raises(M.MpirError):
            M.batch_set_tuning(M.F64, M.F16, u)
    with pytest.raises(M.MpirError):
        M.batch_get_tuning(M.F16, M.F16)          # TW = F16 is not a working precision here
    M.batch_set_tuning(M.F64, M.F16, None)
    assert M.batch_get_tuning(M.F64, M.F16).as_dict() == d0
