"""Projected-gradient block solvers on the GPU (ntf_pgd_update, and ntf_solve with the
inner_solver option) against the FP64 oracle (oracle/pgd.py) on identical inputs."""
import numpy as np
import pytest

import oracle
import synth
from tests.helpers import dev_f32, dev_tensor, ensure_built, rel_fro, to_np

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ntf():
    ensure_built()
    import paper_2001_04321_amd as m
    yield m
    torch.cuda.synchronize()
    assert m.ntf_device_flags() == 0


def _block(seed, I, r, m=80):
    g = np.random.default_rng(seed)
    B = g.random((m, r))
    X = g.random((I, m))
    P = (X @ B).astype(np.float32)
    G = (B.T @ B).astype(np.float32)
    return P, G, g.random((I, r)).astype(np.float32)


@pytest.mark.parametrize("I,r", [(300, 32), (101, 64), (37, 100), (5, 1)])
@pytest.mark.parametrize("accel", [False, True])
def test_block_solver_matches_the_oracle(ntf, I, r, accel):
    P, G, W0 = _block(I + r, I, r)
    W = dev_f32(W0)
    L = ntf.ntf_pgd_update(W, dev_f32(P), dev_f32(G), 50, accel=accel)
    torch.cuda.synchronize()
    G64, P64 = G.astype(np.float64), P.astype(np.float64)
    assert float(L.item()) == pytest.approx(oracle.lipschitz(G64), rel=1e-6)
    solver = oracle.nesterov if accel else oracle.pgd
    ref, steps, _ = solver(W0.astype(np.float64), P64, G64, max_iters=50, tol=0.0)
    # float32 steps against float64 ones: the same steps in numpy float32 set the scale
    err = rel_fro(to_np(W), ref)
    print(f"pgd I={I} r={r} accel={accel} relerr={err:.3e}")
    assert err <= 1e-4
    assert to_np(W).min() >= 0.0


@pytest.mark.parametrize("inner", ["pgd", "nesterov"])
@pytest.mark.parametrize("dims,r,seed", [((30, 20, 25), 5, 1), ((9, 8, 7, 6), 3, 2),
                                         ((40, 35, 30), 40, 3), ((20, 30, 25), 128, 4)])
def test_solve_with_gradient_blocks_matches_the_oracle(ntf, inner, dims, r, seed):
    pr = synth.make_problem(dims, r, snr_db=30.0, data_seed=seed, init_seed=seed + 50)
    T32 = pr.T.astype(np.float32)
    A0 = [a.astype(np.float32) for a in pr.A0]
    Td, T64 = dev_tensor(T32, "f32")
    A = [dev_f32(a) for a in A0]
    iters = 30
    params = ntf.HerParams(inner=inner, inner_tol=0.0, max_inner=50)
    _, tr = ntf.ntf_solve(Td, A, iters, params=params)
    torch.cuda.synchronize()
    ref = oracle.her_solve(T64, [a.astype(np.float64) for a in A0], iters,
                           params=oracle.HERParams(inner=inner, inner_tol=0.0, max_inner=50))
    fh = tr["fhat"].cpu().numpy()
    rs = tr["restart"].cpu().numpy()
    half_norm2 = 0.5 * float(np.sum(T64 * T64))
    prev = ref.fhat0
    for k in range(iters):
        if abs(ref.fhat[k] - prev) < 1e-4 * abs(prev):
            break
        assert bool(rs[k]) == ref.restart[k], k
        # F-hat is a difference of terms of the size of ||T||^2 / 2, which float32 MTTKRPs
        # carry to about 1e-7 relative
        assert abs(fh[k] - ref.fhat[k]) <= 1e-4 * abs(ref.fhat[k]) + 1e-6 * half_norm2, k
        prev = ref.fhat[k]
    assert np.all(tr["sweeps"].cpu().numpy() == 50)
    A_gpu = [to_np(a) for a in A]
    assert min(a.min() for a in A_gpu) >= 0.0
    f_gpu, f_ref = oracle.fit(T64, A_gpu), oracle.fit(T64, ref.factors)
    print(f"{inner} dims={dims} r={r} fit gpu={f_gpu:.6f} oracle={f_ref:.6f}")
    assert abs(f_gpu - f_ref) <= 1e-3 * f_ref


def test_gradient_blocks_reject_a_tolerance_and_the_batched_solver(ntf):
    pr = synth.make_problem((10, 9, 8), 3, snr_db=30.0, data_seed=5, init_seed=6)
    Td, _ = dev_tensor(pr.T.astype(np.float32), "f32")
    A = [dev_f32(a) for a in pr.A0]
    with pytest.raises(ntf.NtfError, match="inner_tol"):
        ntf.ntf_solve(Td, A, 2, params=ntf.HerParams(inner="pgd"))
    with pytest.raises(ntf.NtfError, match="A-HALS"):
        ntf.ntf_solve_batched([Td], [A], 2, params=ntf.HerParams(inner="pgd", inner_tol=0.0))


def test_gradient_blocks_beyond_the_ahals_row_limit(ntf):
    """A block of 13000 rows (more than the resident A-HALS kernel's 12288 at r <= 32):
    projected-gradient blocks (rows are independent) cover it as they cover any block."""
    pr = synth.make_problem((13000, 8, 6), 4, snr_db=30.0, data_seed=8, init_seed=9)
    T32 = pr.T.astype(np.float32)
    A0 = [a.astype(np.float32) for a in pr.A0]
    Td, T64 = dev_tensor(T32, "f32")
    A = [dev_f32(a) for a in A0]
    iters = 5
    params = ntf.HerParams(inner="pgd", inner_tol=0.0, max_inner=50)
    _, tr = ntf.ntf_solve(Td, A, iters, params=params)
    torch.cuda.synchronize()
    ref = oracle.her_solve(T64, [a.astype(np.float64) for a in A0], iters,
                           params=oracle.HERParams(inner="pgd", inner_tol=0.0, max_inner=50))
    half_norm2 = 0.5 * float(np.sum(T64 * T64))
    fh = tr["fhat"].cpu().numpy()
    for k in range(iters):
        assert abs(fh[k] - ref.fhat[k]) <= 1e-4 * abs(ref.fhat[k]) + 1e-6 * half_norm2, k
    f_gpu = oracle.fit(T64, [to_np(a) for a in A])
    assert abs(f_gpu - oracle.fit(T64, ref.factors)) <= 1e-3 * oracle.fit(T64, ref.factors)
