"""Kernel-by-kernel parity of the HIP path (through the C ABI) against the FP64 oracle on
identical inputs (the float32 / bfloat16 values the GPU sees, upcast to float64).

Tolerances (relative Frobenius unless stated):
  MTTKRP <= 1e-5 for both forms (the oracle sees the values the tensor holds: the bf16 form
  rounds only the stored tensor, the factors enter the matrix cores as bf16 hi + lo
  halves), and elementwise |P - P_ref| <= 2e-5 times the sum of the absolute terms of that
  element (float32 accumulation over up to a few hundred sequential adds, and the hi + lo
  split's 2^-18 relative remainder per factor value); the fused all-mode 4-way kernel, whose
  factor blocks are bf16 only, <= 2e-2 (the benchmark spec's bound for the reduced-precision path);
  Gram float64 <= 1e-13, float32 <= 1e-6;
  A-HALS (fixed sweeps) <= 4x the error of a plain numpy float32 run of the same sweeps;
  extrapolation bit-exact (both sides evaluate the same float64 expression, then round);
  F-hat |diff| <= 1e-12 ||T||^2; ||T||^2 <= 1e-13; bf16 cast bit-exact.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.helpers import dev_f32, dev_tensor, elementwise_err, ensure_built, rel_fro, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _lib():
    ensure_built()
    import paper_2001_04321_amd as ntf
    yield ntf
    torch.cuda.synchronize()
    assert ntf.ntf_device_flags() == 0


@pytest.fixture(scope="module")
def ntf(_lib):
    return _lib


# (dims, r): several tiles, ragged tails, odd extents (scalar load path), a unit mode,
# matrices, order 5, wide ranks (two / four / eight 32-column tiles)
MTTKRP_CASES = [
    ((50, 50, 50), 10), ((37, 41, 29), 5), ((3, 4, 5), 3), ((2, 3, 4, 5), 4),
    ((16, 1, 33), 7), ((130, 70, 9), 33), ((5, 200), 64), ((200, 3), 1),
    ((4, 3, 2, 5, 3), 2), ((64, 64, 64), 100), ((20, 30, 40), 250), ((96, 160, 48), 32),
    ((400, 24, 24), 32), ((24, 400, 24), 32), ((24, 24, 400), 32),
]


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("dims,r", MTTKRP_CASES)
def test_mttkrp_matches_oracle(ntf, dims, r, dtype):
    g = np.random.default_rng(hash((dims, r)) % 2**32)
    T = g.random(dims).astype(np.float32)
    A = [g.random((I, r)).astype(np.float32) for I in dims]
    Td, T64 = dev_tensor(T, dtype)
    Ad = [dev_f32(a) for a in A]
    A64 = [a.astype(np.float64) for a in A]
    for n in range(len(dims)):
        P = to_np(ntf.ntf_mttkrp(Td, Ad, n))
        ref = oracle.mttkrp(T64, A64, n)
        err = rel_fro(P, ref)
        ew = elementwise_err(P, ref, ref)
        print(f"mttkrp {dtype} dims={dims} r={r} mode={n} relerr={err:.3e} elementwise={ew:.3e}")
        assert err <= 1e-5, (n, err)
        assert ew <= 2e-5, (n, ew)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_mttkrp_signed_data_and_determinism(ntf, dtype):
    g = np.random.default_rng(3)
    dims, r = (70, 90, 110), 24
    T = g.standard_normal(dims).astype(np.float32)
    A = [g.random((I, r)).astype(np.float32) for I in dims]
    Td, T64 = dev_tensor(T, dtype)
    Ad = [dev_f32(a) for a in A]
    for n in range(3):
        P1 = ntf.ntf_mttkrp(Td, Ad, n)
        P2 = ntf.ntf_mttkrp(Td, Ad, n)
        assert torch.equal(P1, P2)
        ref = oracle.mttkrp(T64, [a.astype(np.float64) for a in A], n)
        # signed data cancels: compare against the scale of the terms, not of the sum
        scale = oracle.mttkrp(np.abs(T64), [a.astype(np.float64) for a in A], n)
        err = np.abs(to_np(P1) - ref).max() / np.abs(scale).max()
        print(f"signed {dtype} mode={n} max error / max scale {err:.3e}")
        assert err <= 1e-6
        assert elementwise_err(to_np(P1), ref, scale) <= 2e-5


# bf16 tensors whose row stride (in the mode under test) is a multiple of 1 MiB: that
# mode runs on the row-slab kernel (one output row per workgroup, u rows in the MFMA M
# dimension). Cases: innermost u mode a multiple of 32 and not (48: a ragged last block),
# v not a multiple of the 64-element chunk (72), r in one and two N tiles (40: a ragged
# second tile), and a 5-way tensor whose slab mode is not the first, with two outer u modes.
SLAB = [((3, 64, 64, 128), 40, 0), ((2, 256, 48, 128), 20, 0), ((2, 256, 256, 72), 24, 0),
        ((2, 3, 64, 64, 128), 8, 1)]


@pytest.mark.parametrize("dims,r,mode", SLAB)
def test_mttkrp_row_slab_modes(ntf, dims, r, mode):
    g = np.random.default_rng(7)
    T = g.random(dims).astype(np.float32)
    A = [g.random((I, r)).astype(np.float32) for I in dims]
    Td, T64 = dev_tensor(T, "bf16")
    Ad = [dev_f32(a) for a in A]
    A64 = [a.astype(np.float64) for a in A]
    P1 = ntf.ntf_mttkrp(Td, Ad, mode)
    P2 = ntf.ntf_mttkrp(Td, Ad, mode)
    assert torch.equal(P1, P2)
    ref = oracle.mttkrp(T64, A64, mode)
    err = rel_fro(to_np(P1), ref)
    ew = elementwise_err(to_np(P1), ref, ref)
    print(f"slab dims={dims} r={r} mode={mode} relerr={err:.3e} elementwise={ew:.3e}")
    assert err <= 1e-5
    assert ew <= 2e-5


@pytest.mark.parametrize("dims,r,dtype,modes", [
    ((70, 90, 110), 24, "f32", (0, 1)), ((70, 90, 110), 24, "bf16", (0, 1, 2)),
    ((70, 90, 110), 24, "f32", (2,)), ((20, 20, 8), 40, "f32", (0, 1, 2)),
    ((9, 8, 7, 6), 5, "f32", (0, 1, 2, 3)), ((60, 50, 40), 70, "bf16", (0, 1)),
    ((5, 7, 128, 128), 40, "bf16", (0, 1, 2, 3)), ((3, 4, 128, 128), 20, "bf16", (0, 1, 2, 3)),
    ((5, 7, 128, 128), 40, "bf16", (0, 2))])
def test_mttkrp_multi(ntf, dims, r, dtype, modes):
    """Several modes with the same factors in one call (3-way: the first two modes through
    Y = T x_3 A_3 when Y is smaller than T; (20, 20, 8) r = 40 is not; 4-way bf16 with
    128 x 128 trailing modes and every mode asked: the fused one-pass kernel, in one and
    two N tiles)."""
    g = np.random.default_rng(5)
    T = g.random(dims).astype(np.float32)
    A = [g.random((I, r)).astype(np.float32) for I in dims]
    Td, T64 = dev_tensor(T, dtype)
    Ad = [dev_f32(a) for a in A]
    A64 = [a.astype(np.float64) for a in A]
    out = ntf.ntf_mttkrp_multi(Td, Ad, modes)
    assert sorted(out) == sorted(modes)
    tol = 1e-5 if dtype == "f32" else 2e-2
    for n, P in out.items():
        err = rel_fro(to_np(P), oracle.mttkrp(T64, A64, n))
        print(f"multi {dtype} dims={dims} r={r} mode={n} relerr={err:.3e}")
        assert err <= tol, (n, err)


def test_mttkrp_multi_full_size_quad128(ntf):
    """The fused all-mode kernel on the 128^4 bf16 r = 64 workload; one row in every
    32-row tile of each mode."""
    pr = synth.workload("quad128_r64_sparse")
    Td, T64 = dev_tensor(pr.T, "bf16")
    A = [a.astype(np.float32) for a in pr.A0]
    del pr
    out = ntf.ntf_mttkrp_multi(Td, [dev_f32(a) for a in A], (0, 1, 2, 3))
    A64 = [a.astype(np.float64) for a in A]
    g = np.random.default_rng(1)
    for n in range(4):
        rows = tile_rows(128, g)
        err = rel_fro(to_np(out[n])[rows], oracle.mttkrp_rows(T64, A64, n, rows))
        print(f"fused quad128 mode={n} rows={rows} relerr={err:.3e}")
        assert err <= 2e-2
    del Td
    torch.cuda.empty_cache()


FULL = [("cube400_r32_corr", "f32"), ("cube400_r32_corr", "bf16"),
        ("quad128_r64_sparse", "bf16"), ("cube512_r50", "f32")]


def tile_rows(I, g, tile=32):
    """One random row in every 32-row tile, plus the first and the last row."""
    rows = {0, I - 1}
    for t0 in range(0, I, tile):
        rows.add(int(g.integers(t0, min(I, t0 + tile))))
    return sorted(rows)


@pytest.mark.parametrize("name,dtype", FULL)
def test_mttkrp_full_size(ntf, name, dtype):
    """Full workload sizes, in the launch configuration the solver uses. 400^3: every row
    (the oracle's full MTTKRP is one library product); 128^4 and 512^3: one row in every
    32-row tile and both ends. Relative Frobenius <= 1e-5 and the elementwise bound."""
    pr = synth.workload(name)
    Td, T64 = dev_tensor(pr.T, dtype)
    A = [a.astype(np.float32) for a in pr.A0]
    del pr
    Ad = [dev_f32(a) for a in A]
    A64 = [a.astype(np.float64) for a in A]
    g = np.random.default_rng(0)
    full = T64.shape[0] == 400
    for n in range(T64.ndim):
        P = to_np(ntf.ntf_mttkrp(Td, Ad, n))
        rows = list(range(T64.shape[n])) if full else tile_rows(T64.shape[n], g)
        ref = oracle.mttkrp(T64, A64, n) if full else oracle.mttkrp_rows(T64, A64, n, rows)
        err = rel_fro(P[rows], ref)
        ew = elementwise_err(P[rows], ref, ref)  # T >= 0 and A >= 0: the terms are >= 0
        print(f"{name} {dtype} mode={n} rows={len(rows)} relerr={err:.3e} elementwise={ew:.3e}")
        assert err <= 1e-5
        assert ew <= 2e-5
    del Td
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dims,r,exclude", [((50, 60, 70), 10, 1), ((130, 7, 200), 33, -1),
                                            ((64, 64, 64, 64), 64, 3), ((3, 5), 1, 0),
                                            ((100, 90), 128, -1)])
def test_gram_hadamard(ntf, dims, r, exclude):
    g = np.random.default_rng(1)
    A = [g.random((I, r)).astype(np.float32) for I in dims]
    G32, G64 = ntf.ntf_gram([dev_f32(a) for a in A], exclude=exclude)
    A64 = [a.astype(np.float64) for a in A]
    ref = oracle.hadamard_gram(A64, exclude) if exclude >= 0 else \
        oracle.hadamard_gram(A64 + [np.ones((1, r))], len(A))
    assert rel_fro(to_np(G64), ref) <= 1e-13
    assert rel_fro(to_np(G32), ref) <= 1e-6


def _hals_f32(W0, P, G, sweeps):
    """Plain float32 numpy A-HALS (calibration of float32 rounding, not the oracle)."""
    W = W0.astype(np.float32).copy()
    P = P.astype(np.float32)
    G = G.astype(np.float32)
    r = W.shape[1]
    for _ in range(sweeps):
        for j in range(r):
            idx = [l for l in range(r) if l != j]
            s = W[:, idx] @ G[idx, j] if idx else 0
            W[:, j] = np.maximum(np.float32(0), P[:, j] - s) / G[j, j] if G[j, j] != 0 else 0
    return W


@pytest.mark.parametrize("dims,r,n,sweeps", [((60, 50, 40), 10, 0, 5), ((400, 30, 30), 32, 0, 8),
                                             ((20, 300, 20), 64, 1, 4), ((25, 25, 25), 3, 2, 10),
                                             ((77, 40, 40), 100, 0, 3), ((10, 9, 8), 1, 1, 2)])
def test_hals_fixed_sweeps(ntf, dims, r, n, sweeps):
    pr = synth.make_problem(dims, r, snr_db=30.0, data_seed=5, init_seed=6)
    A = [a.astype(np.float32) for a in pr.A0]
    T32 = pr.T.astype(np.float32)
    P = oracle.mttkrp(T32.astype(np.float64), [a.astype(np.float64) for a in A], n).astype(np.float32)
    G = oracle.hadamard_gram([a.astype(np.float64) for a in A], n).astype(np.float32)
    Wd = dev_f32(A[n])
    sw = ntf.ntf_hals_update(Wd, dev_f32(P), dev_f32(G), max_sweeps=sweeps, tol=0.0)
    W_gpu = to_np(Wd)
    W_ref, s_ref, _ = oracle.hals(A[n].astype(np.float64), P.astype(np.float64),
                                  G.astype(np.float64), max_sweeps=sweeps, tol=0.0)
    W_np32 = _hals_f32(A[n], P, G, sweeps)
    err_gpu = rel_fro(W_gpu, W_ref)
    err_np = rel_fro(W_np32, W_ref)
    print(f"hals dims={dims} r={r} sweeps={sweeps} gpu={err_gpu:.3e} np32={err_np:.3e}")
    assert int(sw.item()) == s_ref
    assert err_gpu <= max(4 * err_np, 1e-6)
    assert W_gpu.min() >= 0


@pytest.mark.parametrize("rows,r", [(12288, 32), (3072, 128), (3072, 33)])
def test_hals_largest_covered_blocks(ntf, rows, r):
    """The largest blocks the A-HALS kernel covers (256 resident workgroups), with the
    stopping rule at its default tolerance, against the oracle; one row more is refused."""
    g = np.random.default_rng(rows + r)
    # B^(n) has many rows in a real block (a Khatri-Rao product), so G = B^T B is far from
    # singular; a tall B keeps G's conditioning in that range (cond about 1e2-1e3)
    B = g.random((4000, r))
    P = (g.random((rows, 4000)).astype(np.float32) @ B.astype(np.float32)).astype(np.float32)
    G = (B.T @ B).astype(np.float32)
    W0 = g.random((rows, r)).astype(np.float32)
    Wd = dev_f32(W0)
    sw = ntf.ntf_hals_update(Wd, dev_f32(P), dev_f32(G), max_sweeps=10, tol=1e-2)
    W_ref, s_ref, _ = oracle.hals(W0.astype(np.float64), P.astype(np.float64),
                                  G.astype(np.float64), max_sweeps=10, tol=1e-2)
    W_np32 = _hals_f32(W0, P, G, s_ref)
    err_gpu, err_np = rel_fro(to_np(Wd), W_ref), rel_fro(W_np32, W_ref)
    print(f"hals rows={rows} r={r} sweeps={int(sw.item())}/{s_ref} gpu={err_gpu:.3e} "
          f"np32={err_np:.3e}")
    assert int(sw.item()) == s_ref
    # The kernel keeps z = q - W current by rank-one updates (equal to the literal update in
    # exact arithmetic) and re-forms z every 4 sweeps, so up to 4r float32 updates accumulate
    # between refreshes: a forward error of about sqrt(4r) u cond(G) on top of the literal
    # float32 sweeps' (u = 2^-24).
    ev = np.linalg.eigvalsh(G.astype(np.float64))
    bound = 4 * err_np + np.sqrt(4 * r) * 2.0 ** -24 * (ev[-1] / ev[0])
    assert err_gpu <= bound, (err_gpu, bound)
    with pytest.raises(ntf.NtfError, match="EUNSUPPORTED"):
        ntf.ntf_hals_update(dev_f32(np.zeros((rows + 1, r), np.float32)),
                            dev_f32(np.zeros((rows + 1, r), np.float32)), dev_f32(G),
                            max_sweeps=2, tol=0.0)


@pytest.mark.parametrize("rows,r,seed", [(300, 24, 2), (600, 24, 3), (1200, 24, 1),
                                          (2400, 24, 3), (600, 40, 3)])
def test_hals_stopping_rule_workgroup_counts(ntf, rows, r, seed):
    """The stopping rule at the default tolerance for 25, 50, 100 and 200 workgroups (each
    count takes its own form of the rule's cross-workgroup sum: 16, 8 or 4 sweeps per
    round trip, 8 or 16 slot loads per lane) and for 64-lane rows, against the oracle's
    sweep count and iterate. Seeds chosen so that no sweep's ratio lies within 1 % of the
    threshold."""
    g = np.random.default_rng(1000 * rows + r + seed)
    B = g.random((2000, r))
    P = (g.random((rows, 2000)).astype(np.float32) @ B.astype(np.float32)).astype(np.float32)
    G = (B.T @ B).astype(np.float32)
    W0 = g.random((rows, r)).astype(np.float32)
    W_ref, s_ref, deltas = oracle.hals(W0.astype(np.float64), P.astype(np.float64),
                                       G.astype(np.float64), max_sweeps=30, tol=1e-2)
    assert all(abs(d / deltas[0] - 1e-2) > 1e-4 for d in deltas)
    Wd = dev_f32(W0)
    sw = ntf.ntf_hals_update(Wd, dev_f32(P), dev_f32(G), max_sweeps=30, tol=1e-2)
    W_np32 = _hals_f32(W0, P, G, s_ref)
    err_gpu, err_np = rel_fro(to_np(Wd), W_ref), rel_fro(W_np32, W_ref)
    print(f"hals rows={rows} r={r} sweeps={int(sw.item())}/{s_ref} gpu={err_gpu:.3e} "
          f"np32={err_np:.3e}")
    assert int(sw.item()) == s_ref
    # as in test_hals_largest_covered_blocks: the step form's rank-one updates between
    # refreshes add about sqrt(4r) u cond(G) to the literal float32 sweeps' error
    ev = np.linalg.eigvalsh(G.astype(np.float64))
    assert err_gpu <= 4 * err_np + np.sqrt(4 * r) * 2.0 ** -24 * (ev[-1] / ev[0])


def test_hals_stopping_rule_matches_oracle(ntf):
    # seed chosen so that no sweep's delta ratio lies within 1% of the 1e-2 threshold
    pr = synth.make_problem((300, 40, 50), 16, snr_db=30.0, data_seed=29, init_seed=30)
    A = [a.astype(np.float32) for a in pr.A0]
    P = oracle.mttkrp(pr.T.astype(np.float32).astype(np.float64),
                      [a.astype(np.float64) for a in A], 0).astype(np.float32)
    G = oracle.hadamard_gram([a.astype(np.float64) for a in A], 0).astype(np.float32)
    W_ref, s_ref, deltas = oracle.hals(A[0].astype(np.float64), P.astype(np.float64),
                                       G.astype(np.float64), max_sweeps=50, tol=1e-2)
    ratios = [d / deltas[0] for d in deltas]
    # the count is comparable only when no sweep sits on the threshold
    assert all(abs(x - 1e-2) > 1e-4 for x in ratios)
    Wd = dev_f32(A[0])
    sw = ntf.ntf_hals_update(Wd, dev_f32(P), dev_f32(G), max_sweeps=50, tol=1e-2)
    assert int(sw.item()) == s_ref
    assert rel_fro(to_np(Wd), W_ref) <= 1e-4


def test_hals_dead_component_and_unit_sweep(ntf):
    g = np.random.default_rng(9)
    dims, r = (40, 30, 20), 6
    A = [g.random((I, r)).astype(np.float32) for I in dims]
    A[1][:, 4] = 0
    T = g.random(dims).astype(np.float32)
    P = oracle.mttkrp(T.astype(np.float64), [a.astype(np.float64) for a in A], 0).astype(np.float32)
    G = oracle.hadamard_gram([a.astype(np.float64) for a in A], 0).astype(np.float32)
    Wd = dev_f32(A[0])
    sw = ntf.ntf_hals_update(Wd, dev_f32(P), dev_f32(G), max_sweeps=1, tol=1e-2)
    W = to_np(Wd)
    assert int(sw.item()) == 1
    assert np.all(W[:, 4] == 0) and np.all(np.isfinite(W))


def test_norm2_and_cast(ntf):
    g = np.random.default_rng(10)
    for dims in [(101, 33, 7), (64, 64, 64), (5, 3)]:
        T = g.standard_normal(dims).astype(np.float32)
        Td = dev_f32(T)
        n2 = float(ntf.ntf_norm2(Td).item())
        ref = float(np.sum(T.astype(np.float64) ** 2))
        assert abs(n2 - ref) <= 1e-13 * ref
        Tb = ntf.ntf_cast_bf16(Td)
        bits = Tb.view(torch.int16).cpu().numpy().view(np.uint16)
        assert np.array_equal(bits, synth.bf16_bits(T))
        n2b = float(ntf.ntf_norm2(Tb).item())
        refb = float(np.sum(synth.bf16_to_f32(bits).astype(np.float64) ** 2))
        assert abs(n2b - refb) <= 1e-13 * refb


def test_error_surrogate_and_residual(ntf):
    pr = synth.make_problem((60, 50, 40), 8, snr_db=30.0, data_seed=11, init_seed=12)
    T32 = pr.T.astype(np.float32)
    T64 = T32.astype(np.float64)
    A = [a.astype(np.float32) for a in pr.A0]
    A64 = [a.astype(np.float64) for a in A]
    P = oracle.mttkrp(T64, A64, 2).astype(np.float32)
    G = oracle.hadamard_gram(A64, 2)
    normT2 = float(np.sum(T64 ** 2))
    fh = ntf.ntf_error(torch.tensor(normT2, dtype=torch.float64, device="cuda"), dev_f32(P),
                       dev_f32(A[2]), torch.from_numpy(G).cuda())
    ref = oracle.f_hat(normT2, P.astype(np.float64), A64[2], G)
    assert abs(float(fh.item()) - ref) <= 1e-12 * normT2
    res = float(ntf.ntf_residual_norm2(dev_f32(T32), [dev_f32(a) for a in A]).item())
    ref2 = 2 * oracle.objective(T64, A64)
    assert abs(res - ref2) <= 1e-10 * ref2


def test_her_steps_match_oracle(ntf):
    g = np.random.default_rng(13)
    rows, r = [30, 20, 10], 4
    A = [g.random((I, r)).astype(np.float32) for I in rows]
    An = [g.random((I, r)).astype(np.float32) for I in rows]
    Ah = [np.zeros((I, r), np.float32) for I in rows]
    dA, dAn, dAh = [dev_f32(x) for x in A], [dev_f32(x) for x in An], [dev_f32(x) for x in Ah]
    st = ntf.new_state()
    p = ntf.HerParams()
    f0 = torch.tensor(10.0, dtype=torch.float64, device="cuda")
    ntf.ntf_her_step(0, st, p, fhat=f0)
    for b in range(3):
        ntf.ntf_her_step(1, st, p, dA, dAn, dAh, block=b)
        ref = oracle.extrapolate(An[b].astype(np.float64), A[b].astype(np.float64), 0.5)
        assert np.array_equal(to_np(dAh[b]), ref.astype(np.float32).astype(np.float64))
    # decision sequence on crafted F-hat values: 9 (accept), 9.5 (restart), 9.5 (accept)
    b_ref, bb_ref, prev = 0.5, 1.0, 10.0
    for fval in [9.0, 9.5, 9.5, 3.0]:
        ntf.ntf_her_step(2, st, p, dA, dAn, dAh, fhat=torch.tensor(fval, dtype=torch.float64,
                                                                    device="cuda"))
        restart = fval > prev
        b_ref, bb_ref = oracle.update_beta(b_ref, bb_ref, restart, oracle.HERParams())
        prev = fval
        s = ntf.state_dict(st)
        assert s["restart"] == int(restart)
        assert s["beta"] == b_ref and s["beta_bar"] == bb_ref
        for b in range(3):
            want = An[b] if restart else to_np(dAh[b]).astype(np.float32)
            assert np.array_equal(to_np(dA[b]), want.astype(np.float64))
