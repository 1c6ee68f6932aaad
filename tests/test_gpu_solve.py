"""Solver-level parity of ntf_solve (Algorithm 2 on the device, graph-replayed) against the
FP64 oracle on identical float32 inputs.

Restart decisions compare two F-hat values that can differ by less than float32 rounding
of the MTTKRP, so device and oracle trajectories may part after a while (both are valid
runs of the method). What must agree: the decisions while F-hat moves by far more than
rounding, the final fit 1 - ||T - [[A]]|| / ||T|| within 1e-3 relative, nonnegativity,
and a run split by resume must equal an uninterrupted one bit for bit.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.helpers import dev_f32, dev_tensor, ensure_built, to_np

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ntf():
    ensure_built()
    import paper_2001_04321_amd as m
    yield m
    torch.cuda.synchronize()
    assert m.ntf_device_flags() == 0


def _run_gpu(ntf, T, A0, iters, dtype="f32", params=None):
    Td, T64 = dev_tensor(T, dtype)
    A = [dev_f32(a) for a in A0]
    st, tr = ntf.ntf_solve(Td, A, iters, params=params)
    torch.cuda.synchronize()
    return [to_np(a) for a in A], {k: v.cpu().numpy() for k, v in tr.items()}, st, T64


def _fit(T64, A):
    return oracle.fit(T64, A)


@pytest.mark.parametrize("dims,r,seed", [((12, 10, 8), 3, 0), ((30, 20, 25), 5, 1),
                                         ((9, 8, 7, 6), 3, 2), ((40, 35), 4, 3),
                                         ((16, 14, 12, 10), 40, 11),
                                         # 4-way with small (I1 I2 x r) and (I3 I4 x r):
                                         # two tensor passes per iteration (W and V)
                                         ((20, 18, 30, 34), 5, 12), ((33, 7, 16, 40), 8, 13)])
def test_small_problem_trajectory_and_fit(ntf, dims, r, seed):
    pr = synth.make_problem(dims, r, snr_db=30.0, data_seed=seed, init_seed=seed + 50)
    T32 = pr.T.astype(np.float32)
    A0 = [a.astype(np.float32) for a in pr.A0]
    iters = 40
    A_gpu, tr, st, T64 = _run_gpu(ntf, T32, A0, iters)
    ref = oracle.her_solve(T64, [a.astype(np.float64) for a in A0], iters)
    # decisions agree while the F-hat change is far above float32 rounding
    prev = ref.fhat0
    for k in range(iters):
        if abs(ref.fhat[k] - prev) < 1e-4 * abs(prev):
            break
        assert bool(tr["restart"][k]) == ref.restart[k], k
        assert tr["fhat"][k] == pytest.approx(ref.fhat[k], rel=1e-4)
        prev = ref.fhat[k]
    assert min(a.min() for a in A_gpu) >= 0
    f_gpu, f_ref = _fit(T64, A_gpu), _fit(T64, ref.factors)
    print(f"dims={dims} r={r} fit gpu={f_gpu:.6f} oracle={f_ref:.6f}")
    assert abs(f_gpu - f_ref) <= 1e-3 * f_ref


def test_cube50_r10_final_fit(ntf):
    """The 50^3, r = 10, 40 dB workload for 200 outer iterations."""
    pr = synth.workload("cube50_r10")
    T32 = pr.T.astype(np.float32)
    A0 = [a.astype(np.float32) for a in pr.A0]
    A_gpu, tr, st, T64 = _run_gpu(ntf, T32, A0, 200)
    ref = oracle.her_solve(T64, [a.astype(np.float64) for a in A0], 200)
    f_gpu, f_ref = _fit(T64, A_gpu), _fit(T64, ref.factors)
    print(f"cube50 fit gpu={f_gpu:.8f} oracle={f_ref:.8f} restarts gpu={tr['restart'].sum()} "
          f"oracle={sum(ref.restart)}")
    assert abs(f_gpu - f_ref) <= 1e-3 * f_ref
    assert np.all(tr["sweeps"] >= 1) and np.all(tr["sweeps"] <= 50)
    assert np.all(tr["beta"] > 0) and np.all(tr["beta"] <= tr["beta_bar"])
    assert np.all(tr["beta_bar"] <= 1.0)


def test_plain_bcd_is_monotone(ntf):
    pr = synth.make_problem((30, 25, 20), 4, snr_db=30.0, data_seed=4, init_seed=5)
    A_gpu, tr, st, T64 = _run_gpu(ntf, pr.T.astype(np.float32),
                                  [a.astype(np.float32) for a in pr.A0], 30,
                                  params=ntf.HerParams(beta0=0.0))
    f = tr["fhat"]
    assert np.all(tr["beta"] == 0.0)
    assert np.all(np.diff(f) <= 1e-5 * f[:-1])


def test_resume_is_bitwise_identical(ntf):
    pr = synth.make_problem((40, 30, 20), 6, snr_db=30.0, data_seed=6, init_seed=7)
    Td, _ = dev_tensor(pr.T, "f32")
    A1 = [dev_f32(a) for a in pr.A0]
    A2 = [dev_f32(a) for a in pr.A0]
    ntf.ntf_solve(Td, A1, 25)
    st, _ = ntf.ntf_solve(Td, A2, 10)
    ntf.ntf_solve(Td, A2, 15, state=st, resume=True)
    torch.cuda.synchronize()
    for a, b in zip(A1, A2):
        assert torch.equal(a, b)


def test_bf16_tensor_solve_reaches_oracle_fit(ntf):
    pr = synth.make_problem((64, 48, 40), 6, snr_db=30.0, data_seed=8, init_seed=9)
    A0 = [a.astype(np.float32) for a in pr.A0]
    A_gpu, tr, st, Tq = _run_gpu(ntf, pr.T.astype(np.float32), A0, 60, dtype="bf16")
    T64 = pr.T.astype(np.float32).astype(np.float64)
    ref = oracle.her_solve(T64, [a.astype(np.float64) for a in A0], 60)
    f_gpu, f_ref = _fit(T64, A_gpu), _fit(T64, ref.factors)
    print(f"bf16 fit gpu={f_gpu:.6f} oracle={f_ref:.6f}")
    assert abs(f_gpu - f_ref) <= 1e-3 * f_ref


def test_four_way_bf16_two_pass_trajectory(ntf):
    """A bf16 4-way tensor on the two-pass path against the oracle on its bf16 values."""
    pr = synth.make_problem((24, 20, 32, 36), 6, snr_db=30.0, data_seed=14, init_seed=15)
    A0 = [a.astype(np.float32) for a in pr.A0]
    A_gpu, tr, st, Tq = _run_gpu(ntf, pr.T.astype(np.float32), A0, 30, dtype="bf16")
    ref = oracle.her_solve(Tq, [a.astype(np.float64) for a in A0], 30)
    # F-hat is a difference of terms of size ||T||^2, 7e3 times F-hat here: float32 rounding
    # of the MTTKRP moves it by about u ||T||^2 (u = 2^-24), so the tolerance is
    # 1e-4 |F-hat| + 8 u ||T||^2, and decisions are compared while F-hat moves by more
    normT2 = float(np.sum(Tq * Tq))
    prev = ref.fhat0
    checked = 0
    for k in range(30):
        tol = 1e-4 * abs(ref.fhat[k]) + 2.0 ** -21 * normT2
        if abs(ref.fhat[k] - prev) < 2 * tol:
            break
        assert bool(tr["restart"][k]) == ref.restart[k], k
        assert abs(tr["fhat"][k] - ref.fhat[k]) <= tol, (k, tr["fhat"][k], ref.fhat[k])
        prev = ref.fhat[k]
        checked += 1
    f_gpu, f_ref = _fit(Tq, A_gpu), _fit(Tq, ref.factors)
    print(f"4-way bf16 checked {checked} fit gpu={f_gpu:.6f} oracle={f_ref:.6f}")
    assert checked >= 3
    assert abs(f_gpu - f_ref) <= 1e-3 * f_ref
