"""Failure handling through the C ABI, with every kernel exiting normally:

* invalid arguments return NTF_EINVAL (or NTF_EUNSUPPORTED) before anything is enqueued:
  the caller's output buffers keep their contents;
* a non-finite restart surrogate (Sec. 3.1.3: F-hat drives Algorithm 2's restart test)
  raises NTF_FLAG_NONFINITE, restarts, and is not used as the next iteration's reference;
* the A-HALS kernel's bounded cross-workgroup waits (its stopping rule is decided across
  workgroups) give up when the host sets a zero wait limit: the kernel ends, writes its
  iterate and raises NTF_FLAG_WAIT_TIMEOUT.
"""
import ctypes as C
import math

import numpy as np
import pytest

import synth
from tests.helpers import dev_f32, ensure_built

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ntf():
    ensure_built()
    import paper_2001_04321_amd as m
    yield m
    torch.cuda.synchronize()


def _desc(abi, T, order=None, dtype=None, dims=None):
    d = abi.NtfTensor()
    d.order = T.dim() if order is None else order
    d.dtype = (abi.NTF_F32 if T.dtype == torch.float32 else abi.NTF_BF16) if dtype is None else dtype
    for i, s in enumerate(T.shape if dims is None else dims):
        d.dims[i] = int(s)
    d.data = T.data_ptr()
    return d


def test_invalid_arguments_write_nothing(ntf):
    from paper_2001_04321_amd import _abi
    lib = _abi.lib()
    h = ntf.handle().ptr
    g = np.random.default_rng(0)
    dims, r = (20, 30, 40), 5
    T = dev_f32(g.random(dims))
    A = [dev_f32(g.random((I, r))) for I in dims]
    sentinel = 12345.0
    P = torch.full((dims[0], r), sentinel, dtype=torch.float32, device="cuda")
    ptrs = _abi.ptr_array([a.data_ptr() for a in A])
    null_one = _abi.ptr_array([A[0].data_ptr(), None, A[2].data_ptr()])
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    good = _desc(_abi, T)
    bad = {
        "mode": (good, ptrs, r, 3),
        "negative mode": (good, ptrs, r, -1),
        "rank 0": (good, ptrs, 0, 0),
        "rank 257": (good, ptrs, 257, 0),
        "order 1": (_desc(_abi, T, order=1), ptrs, r, 0),
        "order 9": (_desc(_abi, T, order=9, dims=list(dims) + [1] * 5), ptrs, r, 0),
        "dim 0": (_desc(_abi, T, dims=(20, 0, 40)), ptrs, r, 0),
        "NULL factor": (good, null_one, r, 0),
        "dtype": (_desc(_abi, T, dtype=7), ptrs, r, 0),
    }
    for name, (d, pa, rr, mode) in bad.items():
        for fn in (lib.ntf_mttkrp, lib.ntf_mttkrp_noalloc):
            st = fn(h, C.byref(d), pa, rr, mode, P.data_ptr(), stream)
            assert st == _abi.NTF_EINVAL, (name, st, lib.ntf_last_error())
            assert lib.ntf_last_error() != b""
    # ntf_solve: the factors it would overwrite keep their values
    A_keep = [a.clone() for a in A]
    prm = ntf.HerParams().to_c()
    state = ntf.new_state()
    for name, (d, pa, rr) in {"rank": (good, ptrs, 0), "order": (_desc(_abi, T, order=1), ptrs, r),
                               "dims": (_desc(_abi, T, dims=(20, 30, 0)), ptrs, r),
                               "NULL factor": (good, null_one, r),
                               "dtype": (_desc(_abi, T, dtype=3), ptrs, r)}.items():
        st = lib.ntf_solve(h, C.byref(d), rr, pa, C.byref(prm), 3, state.data_ptr(), 0, None,
                           stream)
        assert st == _abi.NTF_EINVAL, (name, st)
    bad_prm = ntf.HerParams(gamma=0.5).to_c()
    assert lib.ntf_solve(h, C.byref(good), r, ptrs, C.byref(bad_prm), 3, state.data_ptr(), 0,
                         None, stream) == _abi.NTF_EINVAL
    # ntf_hals_update: bad rank, rows, sweep count, NULL operands
    W = A[0]
    G = torch.eye(r, dtype=torch.float32, device="cuda")
    sw = torch.full((), -7, dtype=torch.int32, device="cuda")
    for name, args in {"rank 0": (W, P, G, 20, 0, 5), "rank 300": (W, P, G, 20, 300, 5),
                       "rows 0": (W, P, G, 0, r, 5), "sweeps 0": (W, P, G, 20, r, 0),
                       "NULL W": (None, P, G, 20, r, 5), "NULL G": (W, P, None, 20, r, 5)}.items():
        Wp, Pp, Gp, rows, rr, sweeps = args
        st = lib.ntf_hals_update(h, Wp.data_ptr() if Wp is not None else None, Pp.data_ptr(),
                                 Gp.data_ptr() if Gp is not None else None, rows, rr, sweeps,
                                 1e-2, sw.data_ptr(), stream)
        assert st == _abi.NTF_EINVAL, (name, st)
    torch.cuda.synchronize()
    assert bool((P == sentinel).all())
    assert int(sw.item()) == -7
    for a, k in zip(A, A_keep):
        assert torch.equal(a, k)
    assert ntf.ntf_device_flags() == 0


def test_nonfinite_fhat_restarts_and_keeps_the_last_finite_reference(ntf):
    """Crafted F-hat values through the DECIDE step: 9 (accept), NaN (flag, restart; the
    reference stays 9), 9.5: compared with the last finite value 9, so it restarts (a NaN
    reference would accept it, since 9.5 > NaN is false), and becomes the reference."""
    from oracle import HERParams, update_beta
    g = np.random.default_rng(1)
    rows, r = [6, 5, 4], 2
    dA = [dev_f32(g.random((I, r))) for I in rows]
    dAn = [dev_f32(g.random((I, r))) for I in rows]
    dAh = [dev_f32(g.random((I, r))) for I in rows]
    st = ntf.new_state()
    p = ntf.HerParams()
    ntf.ntf_her_step(0, st, p, fhat=torch.tensor(10.0, dtype=torch.float64, device="cuda"))
    b, bb = 0.5, 1.0
    for fval, restart, prev in [(9.0, False, 9.0), (float("nan"), True, 9.0),
                                (9.5, True, 9.5)]:
        ntf.ntf_her_step(2, st, p, dA, dAn, dAh,
                         fhat=torch.tensor(fval, dtype=torch.float64, device="cuda"))
        b, bb = update_beta(b, bb, restart, HERParams())
        s = ntf.state_dict(st)
        assert s["restart"] == int(restart), fval
        assert s["beta"] == b and s["beta_bar"] == bb
        assert s["fhat_prev"] == prev
    assert ntf.ntf_device_flags() & 0x2


def test_nan_in_the_tensor_is_flagged_and_iterates_stay_finite(ntf):
    pr = synth.make_problem((30, 20, 10), 3, snr_db=30.0, data_seed=3, init_seed=4)
    T = pr.T.astype(np.float32)
    T[4, 5, 6] = np.nan
    Td = dev_f32(T)
    A = [dev_f32(a) for a in pr.A0]
    _, tr = ntf.ntf_solve(Td, A, 5)
    torch.cuda.synchronize()
    flags = ntf.ntf_device_flags()
    assert flags & 0x2, flags
    assert not bool(torch.isfinite(tr["fhat"]).any())
    assert bool(tr["restart"].all())
    for a in A:
        assert bool(torch.isfinite(a).all()) and float(a.min()) >= 0.0


def test_zero_wait_limit_forces_the_timeout_path(ntf):
    """A separate handle whose A-HALS waits give up at once: the kernel ends normally, the
    flag is raised; the same call with the default limit raises nothing."""
    h = ntf.Handle(torch.cuda.current_device())
    try:
        g = np.random.default_rng(5)
        rows, r = 400, 32  # 34 workgroups share the stopping rule
        B = g.random((2000, r))
        P = dev_f32(g.random((rows, 2000)) @ B)
        G = dev_f32(B.T @ B)
        W = dev_f32(g.random((rows, r)))
        ntf.ntf_handle_set_wait_limit(0.0, h=h)
        ntf.ntf_hals_update(W, P, G, max_sweeps=50, tol=1e-2, h=h)
        torch.cuda.synchronize()
        assert ntf.ntf_device_flags(h=h) & 0x1
        assert bool(torch.isfinite(W).all()) and float(W.min()) >= 0.0
        pr = synth.make_problem((60, 50, 40), 6, snr_db=30.0, data_seed=6, init_seed=7)
        Td = dev_f32(pr.T)
        A = [dev_f32(a) for a in pr.A0]
        ntf.ntf_solve(Td, A, 3, h=h)
        torch.cuda.synchronize()
        assert ntf.ntf_device_flags(h=h) & 0x1
        ntf.ntf_handle_set_wait_limit(2.0, h=h)
        A = [dev_f32(a) for a in pr.A0]
        ntf.ntf_solve(Td, A, 3, h=h)
        W = dev_f32(g.random((rows, r)))
        ntf.ntf_hals_update(W, P, G, max_sweeps=50, tol=1e-2, h=h)
        torch.cuda.synchronize()
        assert ntf.ntf_device_flags(h=h) == 0
        with pytest.raises(ntf.NtfError, match="EINVAL"):
            ntf.ntf_handle_set_wait_limit(-1.0, h=h)
        assert math.isfinite(float(A[0].sum()))
    finally:
        h.close()
