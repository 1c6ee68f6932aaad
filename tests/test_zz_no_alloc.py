"""The scratch-free MTTKRP entry point (ntf_mttkrp_noalloc) against ntf_mttkrp, through the
C ABI: the same bits in P on two calls in a row, the second on a smaller tensor, in both
tensor forms; the oracle on the same values; a mode whose split partials exceed the
static array is refused with nothing written."""
import numpy as np
import pytest

import oracle
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


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_noalloc_matches_mttkrp_on_two_calls(ntf, dtype):
    g = np.random.default_rng(42)
    # the first tensor has split partials for every mode; the second is smaller, so the
    # array holds stale partials of the first call beyond what the second one writes
    for dims, r in [((96, 130, 72), 24), ((40, 33, 50), 7)]:
        T = g.random(dims).astype(np.float32)
        A = [g.random((I, r)).astype(np.float32) for I in dims]
        Td, T64 = dev_tensor(T, dtype)
        Ad = [dev_f32(a) for a in A]
        A64 = [a.astype(np.float64) for a in A]
        for n in range(len(dims)):
            ref = ntf.ntf_mttkrp(Td, Ad, n)
            out = torch.full((dims[n], r), float("nan"), dtype=torch.float32, device="cuda")
            ntf.ntf_mttkrp_noalloc(Td, Ad, n, out)
            torch.cuda.synchronize()
            assert torch.equal(out, ref), (dims, n)
            err = rel_fro(to_np(out), oracle.mttkrp(T64, A64, n))
            print(f"noalloc {dtype} dims={dims} r={r} mode={n} relerr={err:.2e}")
            assert err <= 1e-5


def test_noalloc_refuses_partials_beyond_the_array(ntf):
    # 512 x 512 x 512 float32 at r = 256: the last mode's split partials (about 128 splits
    # x 512 rows x 256 columns) exceed 4M floats; nothing is launched or written
    dims, r = (512, 512, 512), 256
    T = torch.zeros(dims, dtype=torch.float32, device="cuda")
    A = [torch.zeros((I, r), dtype=torch.float32, device="cuda") for I in dims]
    out = torch.full((dims[2], r), 7.0, dtype=torch.float32, device="cuda")
    with pytest.raises(ntf.NtfError, match="EUNSUPPORTED"):
        ntf.ntf_mttkrp_noalloc(T, A, 2, out)
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
