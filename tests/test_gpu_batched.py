"""Batched solver (ntf_solve_batched: many 3-way problems, each outer iteration of all of
them in a few grouped launches) against the FP64 oracle and against the single-problem
solver, on identical float32 inputs.

Per problem, what must agree with the oracle (as for ntf_solve): restart decisions and
F-hat while F-hat moves by far more than float32 rounding (tests.helpers.check_trajectory), the final fit
1 - ||T - [[A]]|| / ||T|| within 1e-3 relative, nonnegativity; a run split by resume must
equal an uninterrupted one bit for bit; unsupported problems are rejected before launch.
"""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from tests.helpers import check_trajectory, dev_f32, ensure_built, to_np

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_fits.json")
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ntf():
    ensure_built()
    import paper_2001_04321_amd as m
    yield m
    torch.cuda.synchronize()
    assert m.ntf_device_flags() == 0


# shapes with ragged tails, odd sizes, ranks off the 8-column padding, a unit mode
SPECS = [((12, 10, 8), 3), ((30, 20, 25), 5), ((33, 65, 17), 9), ((7, 1, 40), 2),
         ((64, 64, 64), 16), ((50, 31, 70), 20), ((100, 3, 129), 12), ((20, 20, 20), 32)]


def _problems(specs, seed0=0):
    out = []
    for b, (dims, r) in enumerate(specs):
        pr = synth.make_problem(dims, r, snr_db=30.0, data_seed=seed0 + b,
                                init_seed=seed0 + 100 + b)
        out.append((pr.T.astype(np.float32), [a.astype(np.float32) for a in pr.A0]))
    return out


def _run(ntf, probs, iters, resume=False, states=None, dev=None):
    Ts = [torch.from_numpy(T).cuda() for T, _ in probs] if dev is None else dev[0]
    As = [[dev_f32(a) for a in A0] for _, A0 in probs] if dev is None else dev[1]
    states, tr = ntf.ntf_solve_batched(Ts, As, iters, states=states, resume=resume)
    torch.cuda.synchronize()
    return Ts, As, states, tr


def test_batch_matches_oracle_per_problem(ntf):
    probs = _problems(SPECS)
    iters = 30
    Ts, As, states, tr = _run(ntf, probs, iters)
    for b, (T, A0) in enumerate(probs):
        T64 = T.astype(np.float64)
        ref = oracle.her_solve(T64, [a.astype(np.float64) for a in A0], iters)
        fh = tr["fhat"][b].cpu().numpy()
        rs = tr["restart"][b].cpu().numpy()
        checked = check_trajectory(fh, rs, ref, iters, float(np.sum(T64 * T64)))
        assert checked >= 3, b
        A = [to_np(a) for a in As[b]]
        assert min(a.min() for a in A) >= 0
        f_gpu, f_ref = oracle.fit(T64, A), oracle.fit(T64, ref.factors)
        print(f"problem {b} {SPECS[b]}: fit gpu {f_gpu:.6f} oracle {f_ref:.6f}")
        assert abs(f_gpu - f_ref) <= 1e-3 * abs(f_ref)
        st = ntf.batched_state_dict(states, b)
        assert st["k"] == iters and st["nrestarts"] == int(rs.sum())
        sw = tr["sweeps"][b].cpu().numpy()
        assert sw.min() >= 1 and sw.max() <= 50


def test_batch_agrees_with_single_problem_solver(ntf):
    probs = _problems(SPECS[:4], seed0=40)
    iters = 25
    _, As, _, _ = _run(ntf, probs, iters)
    for b, (T, A0) in enumerate(probs):
        T64 = T.astype(np.float64)
        A1 = [dev_f32(a) for a in A0]
        ntf.ntf_solve(torch.from_numpy(T).cuda(), A1, iters)
        torch.cuda.synchronize()
        f_b = oracle.fit(T64, [to_np(a) for a in As[b]])
        f_s = oracle.fit(T64, [to_np(a) for a in A1])
        assert abs(f_b - f_s) <= 1e-3 * abs(f_s)


def test_batch_resume_is_bitwise_continuation(ntf):
    probs = _problems(SPECS[:5], seed0=70)
    _, A_full, st_full, tr_full = _run(ntf, probs, 20)
    Ts, A_half, st, tr1 = _run(ntf, probs, 12)
    _, A_half, st, tr2 = _run(ntf, probs, 8, resume=True, states=st, dev=(Ts, A_half))
    for b in range(len(probs)):
        for a, c in zip(A_full[b], A_half[b]):
            assert torch.equal(a, c), b
        assert torch.equal(tr_full["fhat"][b][12:], tr2["fhat"][b])
        assert ntf.batched_state_dict(st_full, b) == {
            **ntf.batched_state_dict(st, b), "it": ntf.batched_state_dict(st_full, b)["it"]}


def test_batch_graph_replay_is_deterministic(ntf):
    probs = _problems(SPECS[:3], seed0=90)
    _, A1, _, tr1 = _run(ntf, probs, 10)
    _, A2, _, tr2 = _run(ntf, probs, 10)
    for b in range(3):
        assert torch.equal(tr1["fhat"][b], tr2["fhat"][b])
        for a, c in zip(A1[b], A2[b]):
            assert torch.equal(a, c)


def test_batch_rejects_unsupported_problems(ntf):
    from paper_2001_04321_amd import NtfError
    good = _problems([((8, 8, 8), 3)])
    T, A0 = good[0]
    Td = torch.from_numpy(T).cuda()
    As = [dev_f32(a) for a in A0]
    with pytest.raises(NtfError, match="EUNSUPPORTED"):
        ntf.ntf_solve_batched([torch.zeros((300, 4, 4), device="cuda")],
                              [[dev_f32(np.ones((300, 3), np.float32)),
                                dev_f32(np.ones((4, 3), np.float32)),
                                dev_f32(np.ones((4, 3), np.float32))]], 2)
    with pytest.raises(NtfError, match="EUNSUPPORTED"):
        ntf.ntf_solve_batched([Td], [[dev_f32(np.ones((8, 33), np.float32))] * 3], 2)
    with pytest.raises(ValueError, match="3-way"):  # refused by the binding's shape checks
        ntf.ntf_solve_batched([torch.zeros((4, 4, 4, 4), device="cuda")], [As], 2)
    with pytest.raises(NtfError, match="EUNSUPPORTED"):
        ntf.ntf_solve_batched([Td.to(torch.bfloat16)], [As], 2)
    # nothing ran: the factors are untouched
    for a, a0 in zip(As, A0):
        assert np.array_equal(to_np(a), a0)


def test_batch_full_size_sampled_problems(ntf):
    """The 256-problem workload (I_n ~ U{32..160}, r ~ U{5..20}, 30 dB), 200 iterations in
    one launch; 16 problems checked against the oracle's fit (R17) stored by
    tests/golden/make_golden.py: the five largest by cost (I_1 I_2 I_3 r), the smallest, and
    one from each tenth of the cost order."""
    g = json.load(open(GOLDEN)).get("batch256:200")
    if g is None:
        pytest.skip("no stored oracle fits for the batch")
    specs = synth.batch_specs(256)
    prs = [synth.batch_problem(s, b) for b, s in enumerate(specs)]
    probs = [(p.T.astype(np.float32), [a.astype(np.float32) for a in p.A0]) for p in prs]
    del prs
    iters = int(g["iters"])
    _, As, _, tr = _run(ntf, probs, iters)
    assert len(g["fits"]) == 16
    cost = [np.prod(s[:3]) * s[3] for s in specs]
    largest = set(int(i) for i in np.argsort(cost, kind="stable")[-5:])
    assert largest <= set(int(b) for b in g["fits"])
    for key, f_ref in g["fits"].items():
        b = int(key)
        T64 = probs[b][0].astype(np.float64)
        f_gpu = oracle.fit(T64, [to_np(a) for a in As[b]])
        print(f"batch problem {b} {specs[b]}: fit gpu {f_gpu:.6f} oracle {f_ref:.6f}")
        assert abs(f_gpu - f_ref) <= 1e-3 * abs(f_ref)
    for b in range(len(probs)):
        assert min(float(a.min()) for a in As[b]) >= 0
