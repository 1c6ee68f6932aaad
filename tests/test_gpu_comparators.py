"""The paper's comparison algorithms on the GPU against the FP64 oracle
(oracle/comparators.py) on identical inputs: APG (ntf_solve_apg), iBPG (ntf_solve_ibpg)
and Bro's block-wise extrapolation (ntf_solve with scheme "bro", A-HALS blocks).

What must agree: the objective after each iteration and the restart decisions while the
objective moves by far more than float32 rounding, and the final fit within 1e-3
(relative). Iterates are float32 on the GPU, so later iterations may part legitimately."""
import numpy as np
import pytest

import oracle
import synth
from tests.helpers import dev_f32, dev_tensor, ensure_built, to_np

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASES = [((30, 20, 25), 5, 1), ((9, 8, 7, 6), 3, 2), ((40, 35, 30), 12, 3)]


@pytest.fixture(scope="module")
def ntf():
    ensure_built()
    import paper_2001_04321_amd as m
    yield m
    torch.cuda.synchronize()
    assert m.ntf_device_flags() == 0


def _inputs(dims, r, seed):
    pr = synth.make_problem(dims, r, snr_db=30.0, data_seed=seed, init_seed=seed + 50)
    T32 = pr.T.astype(np.float32)
    A0 = [a.astype(np.float32) for a in pr.A0]
    Td, T64 = dev_tensor(T32, "f32")
    return Td, T64, A0


def _compare(f_gpu, f_ref, f0, half_norm2, rs_gpu=None, rs_ref=None, rel=1e-4):
    prev = f0
    for k in range(len(f_ref)):
        if abs(f_ref[k] - prev) < 1e-3 * abs(prev):
            break
        if rs_gpu is not None:
            assert bool(rs_gpu[k]) == bool(rs_ref[k]), k
        assert abs(f_gpu[k] - f_ref[k]) <= rel * abs(f_ref[k]) + 1e-6 * half_norm2, k
        prev = f_ref[k]
    return k


@pytest.mark.parametrize("dims,r,seed", CASES)
def test_apg_matches_the_oracle(ntf, dims, r, seed):
    Td, T64, A0 = _inputs(dims, r, seed)
    A = [dev_f32(a) for a in A0]
    iters = 40
    f_gpu, rs = ntf.ntf_solve_apg(Td, A, iters)
    ref = oracle.apg_solve(T64, [a.astype(np.float64) for a in A0], iters)
    half_norm2 = 0.5 * float(np.sum(T64 * T64))
    k = _compare(f_gpu, ref.objective, ref.f0, half_norm2, rs, ref.restart)
    A_gpu = [to_np(a) for a in A]
    f_g, f_r = oracle.fit(T64, A_gpu), oracle.fit(T64, ref.factors)
    print(f"apg dims={dims} r={r}: {k} iterations compared, restarts {int(rs.sum())} oracle "
          f"{sum(ref.restart)}, fit gpu {f_g:.6f} oracle {f_r:.6f}")
    assert min(a.min() for a in A_gpu) >= 0.0
    assert all(b <= a * (1 + 1e-6) for a, b in zip(f_gpu, f_gpu[1:]))  # restart: monotone
    assert abs(f_g - f_r) <= 1e-3 * f_r


@pytest.mark.parametrize("dims,r,seed", CASES)
def test_ibpg_matches_the_oracle(ntf, dims, r, seed):
    Td, T64, A0 = _inputs(dims, r, seed)
    A = [dev_f32(a) for a in A0]
    iters, inner = 30, 10
    f_gpu = ntf.ntf_solve_ibpg(Td, A, iters, inner_steps=inner)
    ref = oracle.ibpg_solve(T64, [a.astype(np.float64) for a in A0], iters, max_inner=inner,
                            tol=-1.0)
    half_norm2 = 0.5 * float(np.sum(T64 * T64))
    k = _compare(f_gpu, ref.objective, ref.f0, half_norm2)
    A_gpu = [to_np(a) for a in A]
    f_g, f_r = oracle.fit(T64, A_gpu), oracle.fit(T64, ref.factors)
    print(f"ibpg dims={dims} r={r}: {k} iterations compared, fit gpu {f_g:.6f} oracle {f_r:.6f}")
    assert min(a.min() for a in A_gpu) >= 0.0
    assert abs(f_g - f_r) <= 1e-3 * f_r


@pytest.mark.parametrize("dims,r,seed", CASES)
def test_bro_matches_the_oracle(ntf, dims, r, seed):
    Td, T64, A0 = _inputs(dims, r, seed)
    A = [dev_f32(a) for a in A0]
    iters = 40
    st, tr = ntf.ntf_solve(Td, A, iters, params=ntf.HerParams(scheme="bro"))
    torch.cuda.synchronize()
    ref = oracle.bro_solve(T64, [a.astype(np.float64) for a in A0], iters)
    fh = tr["fhat"].cpu().numpy()
    rs = tr["restart"].cpu().numpy()
    beta = tr["beta"].cpu().numpy()
    half_norm2 = 0.5 * float(np.sum(T64 * T64))
    k = _compare(fh, ref.objective, ref.f0, half_norm2, rs, ref.restart)
    # the omega used at iteration k + 1 (trace: the state's beta after iteration k)
    for j in range(min(k, iters - 1)):
        assert beta[j] == pytest.approx(ref.weights[j + 1], rel=1e-12, abs=1e-15), j
    A_gpu = [to_np(a) for a in A]
    f_g, f_r = oracle.fit(T64, A_gpu), oracle.fit(T64, ref.factors)
    print(f"bro dims={dims} r={r}: {k} iterations compared, restarts {int(rs.sum())} oracle "
          f"{sum(ref.restart)}, fit gpu {f_g:.6f} oracle {f_r:.6f}")
    assert abs(f_g - f_r) <= 1e-3 * f_r


def test_comparator_arguments(ntf):
    Td, _, A0 = _inputs((10, 9, 8), 3, 4)
    A = [dev_f32(a) for a in A0]
    with pytest.raises(ntf.NtfError, match="EINVAL"):
        ntf.ntf_solve_apg(Td, A, 2, delta_w=1.0)
    with pytest.raises(ntf.NtfError, match="EINVAL"):
        ntf.ntf_solve_ibpg(Td, A, 2, inner_steps=0)
    with pytest.raises(ntf.NtfError, match="EUNSUPPORTED"):
        ntf.ntf_solve_batched([Td], [A], 2, params=ntf.HerParams(scheme="bro"))
    for a, a0 in zip(A, A0):
        assert np.array_equal(to_np(a), a0)
