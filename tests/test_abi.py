"""C-ABI contract checks that need no GPU: the library loads, exports every function the
header declares, and rejects NULL handles / bad arguments before touching the device."""
import ctypes as C
import os
import re

import pytest

from tests.helpers import ROOT, ensure_built

HEADER = os.path.join(ROOT, "include", "ntf.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ntf_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    ensure_built()
    from paper_2001_04321_amd import _abi
    return _abi.lib()


def test_header_declares_the_hot_path_calls():
    names = _declared()
    for n in ["ntf_mttkrp", "ntf_gram", "ntf_hals_update", "ntf_her_step", "ntf_error",
              "ntf_solve", "ntf_norm2", "ntf_handle_create", "ntf_handle_destroy",
              "ntf_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_covers_every_declared_symbol():
    from paper_2001_04321_amd import _abi
    assert set(_declared()) == set(_abi.SIGNATURES)


def test_version_and_status_strings(lib):
    assert lib.ntf_version().decode().startswith("ntf")
    assert lib.ntf_status_string(1) == b"NTF_EINVAL"
    assert lib.ntf_status_string(4) == b"NTF_EUNSUPPORTED"


def test_null_handle_is_rejected_without_device_work(lib):
    from paper_2001_04321_amd import _abi
    T = _abi.NtfTensor()
    X = _abi.NtfTucker()
    p = _abi.NtfHerParams(0.5, 1.05, 1.01, 1.5, 50, 0, 1e-2)
    calls = [
        lambda: lib.ntf_norm2(None, C.byref(T), None, None),
        lambda: lib.ntf_mttkrp(None, C.byref(T), None, 4, 0, None, None),
        lambda: lib.ntf_gram(None, None, None, 3, 4, -1, None, None, None),
        lambda: lib.ntf_hals_update(None, None, None, None, 10, 4, 50, 1e-2, None, None),
        lambda: lib.ntf_her_step(None, 0, None, C.byref(p), 3, None, 4, None, None, None, 0,
                                 None, None),
        lambda: lib.ntf_error(None, None, None, None, None, 10, 4, None, None),
        lambda: lib.ntf_solve(None, C.byref(T), 4, None, C.byref(p), 10, None, 0, None, None),
        lambda: lib.ntf_residual_norm2(None, C.byref(T), None, 4, None, None),
        lambda: lib.ntf_cast_bf16(None, None, None, 4, None),
        lambda: lib.ntf_mttkrp_autotune(None, C.byref(T), None, 4, 0, None, 3, None, None,
                                        None, None),
        lambda: lib.ntf_tune_import(None, b"f32:4x4x4:mode0:r4 1 4\n"),
        lambda: lib.ntf_mttkrp_noalloc(None, C.byref(T), None, 4, 0, None, None),
        lambda: lib.ntf_handle_set_wait_limit(None, 1.0),
        lambda: lib.ntf_admm_update(None, None, None, None, 10, 4, 50, 1e-2, None, None),
        lambda: lib.ntf_solve_apg(None, C.byref(T), 4, None, 10, 0.9999, None, None, None),
        lambda: lib.ntf_solve_ibpg(None, C.byref(T), 4, None, 10, 50, 0.99, 1.01, None, None),
        lambda: lib.ntf_tucker_mttkrp(None, C.byref(X), None, 4, 0, None, None),
        lambda: lib.ntf_tucker_norm2(None, C.byref(X), None, None),
        lambda: lib.ntf_solve_tucker(None, C.byref(X), 4, None, C.byref(p), 10, None, 0, None,
                                     None),
    ]
    for call in calls:
        assert call() == _abi.NTF_EINVAL
        assert b"handle" in lib.ntf_last_error()
    assert lib.ntf_tune_export(None, None, 0) == -1


def test_handle_create_rejects_bad_pointer(lib):
    from paper_2001_04321_amd import _abi
    assert lib.ntf_handle_create(None, 0) == _abi.NTF_EINVAL


# The binding is the only layer that sees shapes (the ABI takes raw pointers), so it checks
# them before any call; CPU tensors suffice because the checks run before the device ones.
def _cpu(*shape):
    import torch
    return torch.zeros(shape, dtype=torch.float32)


@pytest.mark.parametrize("case", ["short list", "transposed", "other rank", "bad mode",
                                  "bad out"])
def test_binding_rejects_mismatched_factor_shapes(case):
    import paper_2001_04321_amd as ntf
    T = _cpu(5, 6, 7)
    A = [_cpu(5, 3), _cpu(6, 3), _cpu(7, 3)]
    mode, out = 0, None
    if case == "short list":
        A = A[:2]
    elif case == "transposed":
        A[1] = _cpu(3, 6)
    elif case == "other rank":
        A[2] = _cpu(7, 4)
    elif case == "bad mode":
        mode = 3
    elif case == "bad out":
        out = _cpu(6, 3)
    with pytest.raises(ValueError):
        ntf.ntf_mttkrp(T, A, mode, out=out)
    with pytest.raises(ValueError):
        ntf.ntf_mttkrp_noalloc(T, A, mode, out if out is not None else _cpu(5, 3))
    if case in ("short list", "transposed", "other rank"):
        with pytest.raises(ValueError):
            ntf.ntf_solve(T, A, 3)
        with pytest.raises(ValueError):
            ntf.ntf_residual_norm2(T, A)


def test_binding_rejects_mismatched_block_shapes():
    import paper_2001_04321_amd as ntf
    W, P, G = _cpu(10, 4), _cpu(10, 4), _cpu(4, 4)
    with pytest.raises(ValueError):
        ntf.ntf_hals_update(W, _cpu(10, 5), G)
    with pytest.raises(ValueError):
        ntf.ntf_hals_update(W, P, _cpu(5, 5))
    with pytest.raises(ValueError):
        ntf.ntf_pgd_update(W, _cpu(9, 4), G, 5)
    with pytest.raises(ValueError):
        ntf.ntf_error(_cpu(), P, W, _cpu(3, 3).double())
    with pytest.raises(ValueError):
        ntf.ntf_cp_grad(W, P, _cpu(4, 3).double())
    with pytest.raises(ValueError):
        ntf.ntf_gram([_cpu(10, 4), _cpu(8, 3)])
