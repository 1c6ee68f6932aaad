"""Data in Tucker format on the GPU (Appendix A) against the FP64 oracle (oracle/tucker.py)
on identical float32 inputs, and the row-parallel A-HALS blocks that large modes use.

* ntf_tucker_mttkrp: elementwise against oracle.tucker_mttkrp, each element's error scaled
  by the same product on absolute values (the sum of the absolute terms of every stage),
  at 2e-5: the projections and the expansion accumulate in float64, the core's MTTKRP in
  float32 on the matrix cores.
* ntf_tucker_norm2: float64 throughout, 1e-12 relative to the oracle (also for bases without
  orthonormal columns, where it is not ||G||^2).
* ntf_solve_tucker: decisions and F-hat while F-hat moves by far more than float32
  rounding (1e-4 |F-hat| + 8 u ||T||^2, tests.helpers.check_trajectory), and the final fit (by the format's own residual norm, oracle.tucker_relative_
  error, on the host) within 1e-3 relative of the oracle's; the 153 x 238 x 14000 video-
  shaped workload against its stored oracle fit.
* Modes with more rows than the resident A-HALS kernel holds (more than 12288 rows for
  r <= 32) run the row-parallel variant: dense ntf_solve trajectories on such tensors.
"""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from tests.helpers import (ROOT, check_trajectory, dev_f32, dev_tensor, elementwise_err,
                           ensure_built, to_np)

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ntf():
    ensure_built()
    import paper_2001_04321_amd as m
    yield m
    torch.cuda.synchronize()
    assert m.ntf_device_flags() == 0


def _f32(x):
    return np.ascontiguousarray(x, dtype=np.float32)


def _random_tucker(seed, dims, ranks, orthonormal):
    g = np.random.default_rng(seed)
    core = _f32(g.standard_normal(ranks))
    bases = []
    for n, rp in zip(dims, ranks):
        U = g.standard_normal((n, rp))
        if orthonormal:
            U = np.linalg.qr(U)[0]
        bases.append(_f32(U))
    return core, bases


def _check_trajectory(tr, ref, iters, normT2):
    return check_trajectory(tr["fhat"], tr["restart"], ref, iters, normT2)


@pytest.mark.parametrize("dims,ranks,r,orth", [
    ((40, 33, 57), (6, 5, 7), 4, True),
    ((153, 238, 14000), (30, 30, 30), 10, True),
    ((21, 17, 9, 30), (4, 3, 5, 6), 8, False),
    ((300, 64), (20, 9), 40, False),
    ((70, 50, 90), (12, 10, 11), 100, True),
    # outputs r_p r above 2048 (one workgroup per core index), and a long mode whose row
    # chunks outnumber the projection's workgroups (each takes several chunks)
    ((60, 45, 50), (40, 36, 8), 64, False),
    ((300000, 6, 5), (8, 3, 4), 4, True),
])
def test_tucker_mttkrp_matches_oracle(ntf, dims, ranks, r, orth):
    print(f"tucker mttkrp dims={dims} ranks={ranks} r={r}", flush=True)
    core, bases = _random_tucker(sum(dims) + r, dims, ranks, orth)
    g = np.random.default_rng(r)
    A = [_f32(g.random((n, r))) for n in dims]
    c64 = core.astype(np.float64)
    b64 = [U.astype(np.float64) for U in bases]
    a64 = [a.astype(np.float64) for a in A]
    cd, bd, Ad = dev_f32(core), [dev_f32(U) for U in bases], [dev_f32(a) for a in A]
    for n in range(len(dims)):
        P = to_np(ntf.ntf_tucker_mttkrp(cd, bd, Ad, n))
        ref = oracle.tucker_mttkrp(c64, b64, a64, n)
        scale = oracle.tucker_mttkrp(np.abs(c64), [np.abs(U) for U in b64], a64, n)
        err = elementwise_err(P, ref, scale)
        print(f"  mode {n}: elementwise {err:.2e}")
        assert err <= 2e-5, (n, err)


@pytest.mark.parametrize("dims,ranks,orth", [((40, 33, 57), (6, 5, 7), True),
                                             ((21, 17, 9, 30), (4, 3, 5, 6), False),
                                             ((153, 238, 14000), (30, 30, 30), True),
                                             ((5, 300), (5, 7), False)])
def test_tucker_norm2_matches_oracle(ntf, dims, ranks, orth):
    core, bases = _random_tucker(len(dims) * 31 + ranks[0], dims, ranks, orth)
    n2 = float(ntf.ntf_tucker_norm2(dev_f32(core), [dev_f32(U) for U in bases]).item())
    ref = oracle.tucker_norm2(core.astype(np.float64), [U.astype(np.float64) for U in bases])
    assert abs(n2 - ref) <= 1e-12 * ref, (n2, ref)


def test_tucker_binding_rejects_mismatched_shapes(ntf):
    core, bases = _random_tucker(3, (10, 9, 8), (3, 4, 2), True)
    cd = dev_f32(core)
    bd = [dev_f32(U) for U in bases]
    A = [dev_f32(np.ones((n, 3), np.float32)) for n in (10, 9, 8)]
    with pytest.raises(ValueError):
        ntf.ntf_tucker_mttkrp(cd, [bd[0], bd[2], bd[1]], A, 0)
    with pytest.raises(ValueError):
        ntf.ntf_tucker_mttkrp(cd, bd, [A[0], A[2], A[1]], 0)
    with pytest.raises(ValueError):
        ntf.ntf_tucker_mttkrp(cd, bd[:2], A, 0)


@pytest.mark.parametrize("dims,ranks,r,seed,inner", [
    ((30, 25, 400), (6, 5, 7), 4, 0, "ahals"),
    ((20, 16, 12, 50), (5, 4, 4, 6), 3, 1, "ahals"),
    ((40, 30, 13000), (8, 8, 9), 6, 2, "ahals"),   # mode 3 beyond the resident kernel
    ((30, 25, 400), (6, 5, 7), 4, 3, "admm"),
])
def test_solve_tucker_trajectory_and_fit(ntf, dims, ranks, r, seed, inner):
    print(f"solve_tucker dims={dims} ranks={ranks} r={r} inner={inner}", flush=True)
    pr = synth.make_tucker_problem(dims, ranks, r, snr_db=30.0, data_seed=seed,
                                   init_seed=seed + 40)
    core, bases = _f32(pr.core), [_f32(U) for U in pr.bases]
    A0 = [_f32(a) for a in pr.A0]
    iters = 40
    A = [dev_f32(a) for a in A0]
    params = ntf.HerParams(inner=inner)
    _, tr = ntf.ntf_solve_tucker(dev_f32(core), [dev_f32(U) for U in bases], A, iters,
                                 params=params)
    torch.cuda.synchronize()
    tr = {k: v.cpu().numpy() for k, v in tr.items()}
    c64, b64 = core.astype(np.float64), [U.astype(np.float64) for U in bases]
    ref = oracle.tucker_her_solve(c64, b64, [a.astype(np.float64) for a in A0], iters,
                                  oracle.HERParams(inner=inner))
    checked = _check_trajectory(tr, ref, iters, oracle.tucker_norm2(c64, b64))
    A_gpu = [to_np(a) for a in A]
    assert min(a.min() for a in A_gpu) >= 0
    f_gpu = 1.0 - oracle.tucker_relative_error(c64, b64, A_gpu)
    f_ref = 1.0 - oracle.tucker_relative_error(c64, b64, ref.factors)
    print(f"  checked {checked} decisions; fit gpu={f_gpu:.6f} oracle={f_ref:.6f}")
    assert checked >= 3
    assert abs(f_gpu - f_ref) <= 1e-3 * f_ref
    assert np.all(tr["sweeps"] >= 1) and np.all(tr["sweeps"] <= 50)


def test_solve_tucker_video_workload_fit(ntf):
    """153 x 238 x 14000, Tucker ranks 30, CP rank 10, 30 dB, 200 outer iterations, against
    the stored oracle run (tests/golden/oracle_fits.json)."""
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "oracle_fits.json"))).get(
        "tucker_video_r10")
    if g is None:
        pytest.skip("no stored oracle result for tucker_video_r10")
    pr = synth.tucker_workload("tucker_video_r10")
    core, bases = _f32(pr.core), [_f32(U) for U in pr.bases]
    A = [dev_f32(a) for a in pr.A0]
    _, tr = ntf.ntf_solve_tucker(dev_f32(core), [dev_f32(U) for U in bases], A, g["iters"])
    torch.cuda.synchronize()
    fhat = tr["fhat"].cpu().numpy()
    restart = tr["restart"].cpu().numpy()
    # the first iterations, while F-hat falls fast, follow the stored trajectory
    normT2 = oracle.tucker_norm2(core.astype(np.float64), [U.astype(np.float64) for U in bases])
    prev = g["fhat0"]
    for k in range(10):
        tol = 1e-4 * abs(g["fhat"][k]) + 2.0 ** -21 * normT2
        if abs(g["fhat"][k] - prev) < 2 * tol:
            break
        assert abs(fhat[k] - g["fhat"][k]) <= tol, (k, fhat[k], g["fhat"][k])
        prev = g["fhat"][k]
    A_gpu = [to_np(a) for a in A]
    rel = oracle.tucker_relative_error(core.astype(np.float64),
                                       [U.astype(np.float64) for U in bases], A_gpu)
    print(f"tucker video fit gpu={1 - rel:.8f} oracle={g['fit']:.8f} restarts "
          f"gpu={int(restart.sum())} oracle={g['restarts']}")
    assert abs((1 - rel) - g["fit"]) <= 1e-3 * g["fit"]


@pytest.mark.parametrize("dims,r,seed,iters", [((12300, 16, 12), 6, 0, 25),
                                               ((12500, 10, 9), 20, 1, 25),
                                               ((14, 13000, 11), 5, 2, 25),
                                               ((12400, 9, 8), 26, 3, 8),
                                               ((8, 7, 13000), 16, 4, 15)])
def test_dense_solve_with_row_parallel_hals(ntf, dims, r, seed, iters):
    """Dense tensors with a mode beyond the resident A-HALS kernel: the row kernel with the
    exact rank (r = 5, 6, 16) and with 24 and 32 padded columns (r = 20, 26), in the first,
    middle and last mode."""
    print(f"dense row-parallel dims={dims} r={r}", flush=True)
    pr = synth.make_problem(dims, r, snr_db=30.0, data_seed=seed + 70, init_seed=seed + 80)
    T32 = _f32(pr.T)
    A0 = [_f32(a) for a in pr.A0]
    del pr
    Td, T64 = dev_tensor(T32, "f32")
    A = [dev_f32(a) for a in A0]
    _, tr = ntf.ntf_solve(Td, A, iters)
    torch.cuda.synchronize()
    tr = {k: v.cpu().numpy() for k, v in tr.items()}
    ref = oracle.her_solve(T64, [a.astype(np.float64) for a in A0], iters)
    checked = _check_trajectory(tr, ref, iters, float(np.sum(T64 * T64)))
    A_gpu = [to_np(a) for a in A]
    f_gpu, f_ref = oracle.fit(T64, A_gpu), oracle.fit(T64, ref.factors)
    print(f"  checked {checked}; fit gpu={f_gpu:.6f} oracle={f_ref:.6f}")
    assert checked >= 3
    assert abs(f_gpu - f_ref) <= 1e-3 * f_ref
    assert min(a.min() for a in A_gpu) >= 0


def test_row_parallel_hals_limits_are_refused(ntf):
    """Beyond the resident kernel's rows the row-parallel variant needs r <= 32 and at most
    64 sweeps; other solves are refused, not truncated."""
    Td = dev_f32(np.ones((12300, 3, 2), np.float32))
    A = [dev_f32(np.ones((n, 33), np.float32)) for n in (12300, 3, 2)]
    with pytest.raises(ntf.NtfError, match="EUNSUPPORTED"):
        ntf.ntf_solve(Td, A, 1)
    A = [dev_f32(np.ones((n, 4), np.float32)) for n in (12300, 3, 2)]
    with pytest.raises(ntf.NtfError, match="EUNSUPPORTED"):
        ntf.ntf_solve(Td, A, 1, params=ntf.HerParams(max_inner=65))
