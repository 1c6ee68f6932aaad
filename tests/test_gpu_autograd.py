"""Autograd loss ||T - [[A]]||_F^2 with the hand-written backward (through the C ABI)
against the FP64 oracle and FP64 central finite differences on identical inputs.

Tolerances: forward |dL| <= 1e-6 ||T||^2 (float32 MTTKRP inside a float64 Gram trick);
gradient vs the oracle gradient <= 1e-5 relative Frobenius (float32 tensor), <= 2e-2
(bfloat16 tensor); gradient vs FP64 central differences <= 1e-4 relative Frobenius.
"""
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


def _problem(dims, r, seed):
    g = np.random.default_rng(seed)
    A_true = [g.random((I, r)) for I in dims]
    T = oracle.kruskal(A_true) + 0.05 * g.standard_normal(dims)
    A = [g.random((I, r)).astype(np.float32) for I in dims]
    return T.astype(np.float32), A


def _loss_and_grads(ntf, Td, A, upstream=1.0):
    Ad = [dev_f32(a).requires_grad_(True) for a in A]
    L = ntf.ntf_loss(Td, Ad)
    (L * upstream).backward()
    return float(L.item()), [to_np(a.grad) for a in Ad]


CASES = [((24, 24, 24), 4, 0), ((30, 20, 25), 6, 1), ((6, 7, 8, 5), 3, 2), ((40, 50), 5, 3),
         ((33, 17, 65), 12, 4)]


@pytest.mark.parametrize("dims,r,seed", CASES)
def test_loss_and_gradient_match_oracle(ntf, dims, r, seed):
    T, A = _problem(dims, r, seed)
    Td, T64 = dev_tensor(T, "f32")
    A64 = [a.astype(np.float64) for a in A]
    L, grads = _loss_and_grads(ntf, Td, A)
    L_ref = oracle.cp_loss(T64, A64)
    _, G_ref = oracle.cp_loss_grad(T64, A64)
    nt2 = float(np.sum(T64 * T64))
    print(f"dims={dims} r={r} loss={L:.10e} ref={L_ref:.10e} |dL|/|T|^2={abs(L - L_ref) / nt2:.2e}")
    assert abs(L - L_ref) <= 1e-6 * nt2
    for n, (g, gr) in enumerate(zip(grads, G_ref)):
        err = rel_fro(g, gr)
        print(f"  grad mode {n}: relerr {err:.3e}")
        assert err <= 1e-5


def test_gradient_matches_central_differences(ntf):
    """FP64 central differences of the oracle loss at the float32 point the GPU sees
    (24^3, r = 4, step 1e-6 max(1, |x|))."""
    pr = synth.workload("cube24_r4")
    T = pr.T.astype(np.float32)
    A = [a.astype(np.float32) for a in pr.A0]
    Td, T64 = dev_tensor(T, "f32")
    _, grads = _loss_and_grads(ntf, Td, A)
    A64 = [a.astype(np.float64) for a in A]
    for n in range(3):
        fd = np.zeros_like(A64[n])
        for idx in np.ndindex(*A64[n].shape):
            x = A64[n][idx]
            h = 1e-6 * max(1.0, abs(x))
            Ap = [a.copy() for a in A64]
            Am = [a.copy() for a in A64]
            Ap[n][idx] = x + h
            Am[n][idx] = x - h
            fd[idx] = (oracle.cp_loss(T64, Ap) - oracle.cp_loss(T64, Am)) / (2 * h)
        err = rel_fro(grads[n], fd)
        print(f"mode {n}: GPU gradient vs central differences relerr {err:.3e}")
        assert err <= 1e-4


def test_upstream_gradient_scales_and_partial_requires_grad(ntf):
    T, A = _problem((20, 21, 22), 5, 7)
    Td, _ = dev_tensor(T, "f32")
    _, g1 = _loss_and_grads(ntf, Td, A, 1.0)
    _, g3 = _loss_and_grads(ntf, Td, A, -2.5)
    for a, b in zip(g1, g3):
        np.testing.assert_allclose(b, -2.5 * a, rtol=1e-6, atol=0)
    # only one factor requires a gradient
    Ad = [dev_f32(a) for a in A]
    Ad[1].requires_grad_(True)
    ntf.ntf_loss(Td, Ad).backward()
    assert Ad[0].grad is None and Ad[2].grad is None
    np.testing.assert_allclose(to_np(Ad[1].grad), g1[1], rtol=1e-6, atol=0)


def test_bf16_tensor_gradient(ntf):
    T, A = _problem((48, 40, 36), 8, 11)
    Td, T64 = dev_tensor(T, "bf16")
    A64 = [a.astype(np.float64) for a in A]
    L, grads = _loss_and_grads(ntf, Td, A)
    L_ref = oracle.cp_loss(T64, A64)
    assert abs(L - L_ref) <= 2e-2 * float(np.sum(T64 * T64))
    for g, gr in zip(grads, oracle.cp_loss_grad(T64, A64)[1]):
        assert rel_fro(g, gr) <= 2e-2


def test_cp_grad_kernel_alpha_and_null_scale(ntf):
    g = np.random.default_rng(3)
    A = g.random((37, 9)).astype(np.float32)
    P = g.random((37, 9)).astype(np.float32)
    G = g.random((9, 9))
    G = G + G.T
    out = to_np(ntf.ntf_cp_grad(dev_f32(A), dev_f32(P), torch.from_numpy(G).cuda(), None, 1.0))
    ref = A.astype(np.float64) @ G - P.astype(np.float64)
    assert rel_fro(out, ref) <= 1e-7


def test_autograd_full_size_sampled_rows(ntf):
    """512^3, r = 50 (float32): loss and gradient rows sampled against the oracle."""
    pr = synth.workload("cube512_r50")
    Td, T64 = dev_tensor(pr.T, "f32")
    A = [a.astype(np.float32) for a in pr.A0]
    A64 = [a.astype(np.float64) for a in A]
    L, grads = _loss_and_grads(ntf, Td, A)
    nt2 = float(np.sum(T64 * T64))
    L_ref = oracle.cp_loss(T64, A64)
    print(f"512^3 r=50: loss {L:.10e} ref {L_ref:.10e}")
    assert abs(L - L_ref) <= 1e-6 * nt2
    rng = np.random.default_rng(0)
    for n in range(3):
        rows = sorted(set([0, 511] + list(rng.integers(0, 512, 3))))
        P = oracle.mttkrp_rows(T64, A64, n, rows)
        G = oracle.hadamard_gram(A64, n)
        ref = 2.0 * (A64[n][rows] @ G - P)
        err = rel_fro(grads[n][rows], ref)
        print(f"  mode {n} rows {rows}: relerr {err:.3e}")
        assert err <= 1e-5
    del Td
    torch.cuda.empty_cache()
