"""Final fits of ntf_solve on the full-size synthetic workloads against the FP64 oracle's
stored results (tests/golden/oracle_fits.json, written by tests/golden/make_golden.py,
which calls only the oracle).

* 400^3, r = 32, correlated factors, 30 dB, 500 outer iterations: the float32 tensor and
  its bfloat16 copy; both fits are taken against the float32 tensor the copy was made
  from, and must be within 1e-3 (relative) of the oracle's fit on the float32 values.
* 128^4, r = 64, 30 % zeroed factor entries, 20 dB, clipped, stored in bfloat16: the
  trajectory of 20 outer iterations on a float32 copy of the bfloat16 values against a
  stored 20-iteration oracle run on the same values (F-hat, decisions, fit), the bf16
  form's first iterations, and both forms' fits after 200 outer iterations against the
  oracle's (two-sided).
The final fits are computed on the host by the oracle's explicit residual (float64), and
the device's ntf_residual_norm2 is checked against it at these full sizes.
"""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from tests.helpers import ROOT, dev_f32, dev_tensor, ensure_built

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLDEN = os.path.join(ROOT, "tests", "golden", "oracle_fits.json")


def _golden(key):
    g = json.load(open(GOLDEN)).get(key)
    if g is None:
        pytest.skip(f"no stored oracle result for {key}")
    return g


@pytest.fixture(scope="module")
def ntf():
    ensure_built()
    import paper_2001_04321_amd as m
    yield m
    torch.cuda.synchronize()
    assert m.ntf_device_flags() == 0


@pytest.fixture(scope="module")
def cube400():
    pr = synth.workload("cube400_r32_corr")
    T32 = pr.T.astype(np.float32)
    A0 = [a.astype(np.float32) for a in pr.A0]
    del pr
    Td32 = torch.from_numpy(T32).cuda()
    del T32
    yield Td32, A0


def _relerr(ntf, Tref, A, host=False):
    """Explicit relative error ||T - [[A]]|| / ||T|| of the final factors: on the device
    (ntf_residual_norm2), or with host=True by the oracle on the host (float64), after
    checking that the device value agrees with it to 1e-9 relative."""
    res = float(ntf.ntf_residual_norm2(Tref, A).item()) ** 0.5
    rel = res / float(ntf.ntf_norm2(Tref).item()) ** 0.5
    if not host:
        return rel
    T64 = Tref.float().cpu().double().numpy()
    rel_host = oracle.relative_error(T64, [a.cpu().double().numpy() for a in A])
    del T64
    assert abs(rel - rel_host) <= 1e-9 * rel_host, (rel, rel_host)
    return rel_host


@pytest.mark.parametrize("form", ["f32", "bf16"])
def test_cube400_r32_corr_final_fit(ntf, cube400, form):
    g = _golden("cube400_r32_corr")
    Td32, A0 = cube400
    Td = Td32 if form == "f32" else ntf.ntf_cast_bf16(Td32)
    A = [dev_f32(a) for a in A0]
    _, tr = ntf.ntf_solve(Td, A, g["iters"])
    torch.cuda.synchronize()
    rel = _relerr(ntf, Td32, A, host=True)
    fit, fit_ref = 1.0 - rel, g["fit"]
    print(f"cube400 {form}: relerr {rel:.7f} oracle {g['relerr']:.7f}; restarts "
          f"{int(tr['restart'].sum().item())} oracle {g['restarts']}")
    assert min(float(a.min().item()) for a in A) >= 0.0
    assert abs(fit - fit_ref) <= 1e-3 * fit_ref


def _quad128(ntf, iters, dtype, host=False):
    """Solve the 128^4 workload from its bf16 values, held as bf16 or as float32."""
    pr = synth.workload("quad128_r64_sparse")
    A0 = [a.astype(np.float32) for a in pr.A0]
    Td, T64 = dev_tensor(pr.T, "bf16")
    del pr
    if dtype == "f32":
        Td = torch.from_numpy(T64.astype(np.float32)).cuda()
    del T64
    A = [dev_f32(a) for a in A0]
    _, tr = ntf.ntf_solve(Td, A, iters)
    torch.cuda.synchronize()
    rel = _relerr(ntf, Td, A, host=host)
    assert min(float(a.min().item()) for a in A) >= 0.0
    return rel, tr["fhat"].cpu().numpy(), tr["restart"].cpu().numpy()


def test_quad128_r64_sparse_trajectory(ntf):
    """20 outer iterations on the float32 copy of the bf16 values (exactly the oracle's
    input, float32 MTTKRP): every F-hat, every decision, and the fit. F-hat is a difference
    of terms of the size of ||T||^2 / 2 (about F-hat_0 here) that the float32 MTTKRP
    carries to about 1e-7 relative, so F-hat agrees to 1e-6 F-hat_0 absolute."""
    g = _golden("quad128_r64_sparse:bf16:20")
    rel, fh, rs = _quad128(ntf, g["iters"], "f32")
    dev = np.abs(fh - np.asarray(g["fhat"]))
    print(f"quad128 f32 20 iterations: relerr {rel:.8f} oracle {g['relerr']:.8f}; max F-hat "
          f"deviation {dev.max() / g['fhat0']:.2e} of F-hat_0")
    assert dev.max() <= 1e-6 * g["fhat0"]
    ref_restart = np.diff(np.concatenate([[g["fhat0"]], g["fhat"]])) > 0
    assert np.array_equal(rs.astype(bool), ref_restart)
    assert abs(rel - g["relerr"]) <= 1e-5 * g["relerr"]


def test_quad128_r64_sparse_bf16_first_iterations(ntf):
    """20 outer iterations of the bf16 form. Its MTTKRP rounds only the stored tensor, whose
    values are the oracle's input, so the first F-hat values agree with the oracle's to
    1e-5 F-hat_0 (float32 accumulation), and the fit after 20 iterations is within 1e-3 of
    the oracle's (two-sided)."""
    g = _golden("quad128_r64_sparse:bf16:20")
    rel, fh, rs = _quad128(ntf, g["iters"], "bf16")
    dev = np.abs(fh - np.asarray(g["fhat"]))
    print(f"quad128 bf16 20 iterations: relerr {rel:.7f} oracle {g['relerr']:.7f}; restarts "
          f"{int(rs.sum())} oracle {g['restarts']}; F-hat deviation per iteration / F-hat_0 "
          f"{np.array2string(dev / g['fhat0'], precision=2)}")
    for k in range(3):
        assert dev[k] <= 1e-5 * g["fhat0"], k
        assert not rs[k]
    assert abs((1.0 - rel) - g["fit"]) <= 1e-3 * g["fit"]


def test_quad128_r64_sparse_final_fit(ntf):
    """200 outer iterations, the float32 copy of the bf16 values (the oracle's input) and
    the bf16 form: both final fits within 1e-3 (relative) of the oracle's (R17)."""
    g = _golden("quad128_r64_sparse:bf16")
    rel32, _, rs32 = _quad128(ntf, g["iters"], "f32", host=True)
    rel16, _, rs16 = _quad128(ntf, g["iters"], "bf16", host=True)
    print(f"quad128 {g['iters']} iterations: relerr f32 {rel32:.7f}, bf16 {rel16:.7f}, oracle "
          f"{g['relerr']:.7f}; restarts {int(rs32.sum())}, {int(rs16.sum())}, oracle "
          f"{g['restarts']}")
    assert abs((1.0 - rel32) - g["fit"]) <= 1e-3 * g["fit"]
    assert abs((1.0 - rel16) - g["fit"]) <= 1e-3 * g["fit"]
