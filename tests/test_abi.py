"""The C ABI library loads and exports every declared symbol; argument
validation returns before any device call (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2410_22500_amd", "libhsn.so")
HDR = os.path.join(ROOT, "include", "hsn.h")


def _declared():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hsn_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("libhsn.so not built")
    return C.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert "hsn_subspace_nmf" in names and "hsn_project" in names
    for n in names:
        assert hasattr(lib, n), n


def test_null_context_is_invalid_arg(lib):
    v = C.c_void_p
    lib.hsn_last_error.restype = C.c_char_p
    assert lib.hsn_version() >= 100
    assert lib.hsn_create(None, 0) == 1
    assert lib.hsn_normalize(None, *([v()] * 15)) == 1
    assert lib.hsn_subspace_nmf(None, v(), C.c_int64(0), v(), C.c_int64(0), C.c_int64(1), C.c_int64(1),
                                v(), v(), v(), v(), v()) == 1
    assert lib.hsn_project(None, v(), v(), v(), C.c_float(1), C.c_float(0), v()) == 1
    assert lib.hsn_backproject(None, v(), v(), v(), C.c_float(1), C.c_float(0), v()) == 1
    assert lib.hsn_cgls(None, v(), v(), v(), 1, v(), v()) == 1
    assert lib.hsn_mbir(None, v(), v(), v(), v(), v(), C.c_double(1.2), C.c_double(1.0), 1, 1, v()) == 1
    assert lib.hsn_fhr_step(None, v(), v(), 0, v(), 0, C.c_float(1), v(), C.c_int64(0), v(), v(), v(), v(), v(),
                            v(), 0, v(), C.c_int64(0), C.c_int64(0), C.c_int64(0), C.c_int64(0), v(),
                            C.c_int64(0), v()) == 1
    assert lib.hsn_rehydrate(None, v(), v(), C.c_int64(1), C.c_int64(1), 1, C.c_int64(0), C.c_int64(1),
                             C.c_int64(0), C.c_int64(1), v(), C.c_int64(1), v()) == 1
    assert lib.hsn_last_error(None) == b"null context"


def test_mlp_entry_points_validate_on_host(lib):
    v = C.c_void_p
    lib.hsn_mlp_n_params.restype = C.c_int64
    # 256*128 + 128 + 128*128 + 128 + 128*K + K parameters
    assert lib.hsn_mlp_n_params(4) == 49924
    assert lib.hsn_mlp_n_params(1) == 49408 + 129
    assert lib.hsn_mlp_n_params(0) == -1 and lib.hsn_mlp_n_params(9) == -1
    lib.hsn_mlp_k.argtypes = [v]
    assert lib.hsn_mlp_k(None) == -1
    assert lib.hsn_mlp_create(None, v(), 4, 1, v()) == 1
    assert lib.hsn_mlp_train(None, v(), v(), v(), C.c_int64(1), v(), v(), v()) == 1
    assert lib.hsn_mlp_infer(None, v(), v(), C.c_int64(0), C.c_int64(0), C.c_int64(1), v(), v()) == 1
    assert lib.hsn_canonicalize(None, v(), C.c_int64(1), v(), C.c_int64(1), 1, v(), v()) == 1
    lib.hsn_mlp_destroy(None)
