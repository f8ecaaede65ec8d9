"""CPU-side tests of the C-ABI library: it loads, exports every symbol the
header declares, and its host logic (rule validation and compilation, term
loading, call-order and size checks) behaves as documented -- no device
call is made."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "trs.h")


def _lib():
    from paper_2009_07174_amd import trs as T
    return T


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(trs_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_four_calls():
    names = declared_functions()
    for n in ("trs_load_rules", "trs_load_terms", "trs_normalize", "trs_read_nf"):
        assert n in names


def test_library_exports_every_declared_symbol():
    T = _lib()
    lib = ctypes.CDLL(T.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(declared_functions()) <= set(T.EXPORTS)


def test_status_strings():
    T = _lib()
    for code in range(0, -10, -1):
        assert T._lib.trs_status_str(code)
    assert b"unknown" in T._lib.trs_status_str(-99)


def test_device_bytes_arithmetic():
    T = _lib()
    b2 = T.trs_device_bytes(1 << 20, 2)
    b3 = T.trs_device_bytes(1 << 20, 3)
    assert b3 - b2 >= (1 << 20) * 4 * 2   # pool args and their initial image
    assert T.trs_device_bytes(1, 2) == -1
    assert T.trs_device_bytes(1 << 20, 9) == -1


def _ctx(pool=1 << 12, A=0):
    T = _lib()
    c = T.Context(pool, A, torch_memory=False)
    return T, c


def test_rule_validation_errors():
    from trs_workloads import parse_trs
    T, c = _ctx()
    cases = {
        "lhs variable": "sym f/1 a/0\nvar X\neqn X = a\n",
        "rhs var not in lhs": "sym f/1 a/0\nvar X Y\neqn f(X) = Y\n",
        "not left-linear": "sym f/2 a/0\nvar X\neqn f(X, X) = a\n",
    }
    for what, text in cases.items():
        with pytest.raises(T.TRSError) as e:
            c.load_trs(parse_trs(text))
        assert e.value.code == T.TRS_E_RULE, what
    c.close()


def test_malformed_rule_code_rejected():
    from trs_workloads import systems
    T, c = _ctx()
    arity, off, code = systems.peano().encode_rules()
    bad = code.copy()
    bad[off[1] - 1] = 2          # rhs of rule 0 becomes plus(...) without operands
    with pytest.raises(T.TRSError) as e:
        c.load_rules(arity, off, bad)
    assert e.value.code == T.TRS_E_RULE
    bad = code.copy()
    bad[0] = 99                  # unknown symbol
    with pytest.raises(T.TRSError):
        c.load_rules(arity, off, bad)
    c.close()


def test_maxarity_limit():
    from trs_workloads import systems
    T = _lib()
    c = T.Context(1 << 12, 2, torch_memory=False)
    with pytest.raises(T.TRSError) as e:
        c.load_trs(systems.msort())   # merge2 has arity 3
    assert e.value.code == T.TRS_E_RULE
    c.close()


def test_table_limits():
    from trs_workloads import parse_trs
    T, c = _ctx()
    big = "sym f/1 g/1 a/0\nvar X\neqn f(" + "g(" * 9 + "X" + ")" * 9 + ") = a\n"
    with pytest.raises(T.TRSError) as e:
        c.load_trs(parse_trs(big))
    assert e.value.code == T.TRS_E_LIMIT
    c.close()


def test_call_order_and_term_errors():
    from trs_workloads import systems
    T, c = _ctx(pool=64)
    trs = systems.peano()
    # terms before rules: the context does not exist yet in the binding, so
    # create it through load_rules first and then misuse the order
    c.load_trs(trs)
    with pytest.raises(T.TRSError) as e:
        c.normalize()
    assert e.value.code == T.TRS_E_STATE
    with pytest.raises(T.TRSError) as e:
        c.read_nf(0)
    assert e.value.code == T.TRS_E_STATE
    with pytest.raises(T.TRSError) as e:
        c.load_terms(np.array([0, 2], np.int64), np.array([1, -1], np.int32))
    assert e.value.code == T.TRS_E_TERM
    with pytest.raises(T.TRSError) as e:
        c.load_terms(np.array([0, 2], np.int64), np.array([2, 0], np.int32))  # plus(0, ?)
    assert e.value.code == T.TRS_E_TERM
    with pytest.raises(T.TRSError) as e:   # 65 nodes do not fit in 64 slots
        c.load_term_list([np.array([1] * 64 + [0], np.int32)])
    assert e.value.code == T.TRS_E_POOL
    c.load_term_list([trs.encode("plus(S(0), S(0))")])
    bad_opts = T.Options(block=100)
    with pytest.raises(T.TRSError) as e:
        c.normalize(bad_opts)
    assert e.value.code == T.TRS_E_ARG
    with pytest.raises(T.TRSError) as e:
        c.normalize(T.Options(nodes_per_thread=3))
    assert e.value.code == T.TRS_E_ARG
    # the frontier modes' walk and continuation bounds and the placement
    # share are range-checked before any device work
    for bad in (dict(nf_walk=-2), dict(nf_walk_wide=-5), dict(cont_passes=-2),
                dict(cont_passes_wide=1 << 21), dict(place_fresh=101), dict(place_fresh=-1)):
        with pytest.raises(T.TRSError) as e:
            c.normalize(T.Options(mode=T.TRS_MODE_FRONTIER, **bad))
        assert e.value.code == T.TRS_E_ARG, bad
    c.close()


def test_normalize_without_gpu_reports_hip_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from trs_workloads import systems
    T, c = _ctx()
    trs = systems.peano()
    c.load_trs(trs)
    c.load_term_list([trs.encode("plus(S(0), S(0))")])
    with pytest.raises(T.TRSError) as e:
        c.normalize()
    assert e.value.code == T.TRS_E_HIP
    c.close()


def test_noalloc_eval_rejects_oversized_batches_on_the_host():
    # the size checks come before any device call
    T = _lib()
    n_sym = 3
    P = T.trs_mlp_param_count(n_sym)
    w = np.zeros(P, np.uint16)
    rec = np.zeros(T.TRS_MLP_NOALLOC_MAX_RECORDS + 1, np.uint64)
    with pytest.raises(T.TRSError) as e:
        T.trs_mlp_eval_noalloc(n_sym, w, rec)
    assert e.value.code == T.TRS_E_LIMIT
    with pytest.raises(T.TRSError) as e:
        T.trs_mlp_eval_noalloc(n_sym, w, rec[:0])
    assert e.value.code == T.TRS_E_ARG
