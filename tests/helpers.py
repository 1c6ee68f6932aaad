"""Shared helpers of the test suite (input marshalling, error measures, library build)."""
import os

import numpy as np

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2001_04321_amd", "libntf.so")


def ensure_built():
    """Build libntf.so if nothing is built yet (tests load what is built)."""
    if not os.path.exists(LIB):
        from paper_2001_04321_amd import build
        build.build(verbose=False)


def rel_fro(x, ref) -> float:
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref.ravel())
    return float(np.linalg.norm((x - ref).ravel()) / (den if den > 0 else 1.0))


def elementwise_err(x, ref, scale) -> float:
    """max |x - ref| / scale over the elements (scale: the sum of the absolute terms of
    each element, e.g. the MTTKRP of |T| with |A|; zero-scale elements must match exactly)."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.abs(np.asarray(scale, dtype=np.float64))
    d = np.abs(x - ref)
    if np.any(d[scale == 0] != 0):
        return float("inf")
    return float(np.max(np.where(scale > 0, d / np.where(scale > 0, scale, 1.0), 0.0)))


def dev_f32(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def dev_tensor(T, dtype: str):
    """Device copy of T in float32 or bfloat16 and the float64 values it holds."""
    import torch
    T32 = np.ascontiguousarray(T, dtype=np.float32)
    if dtype == "f32":
        return torch.from_numpy(T32).cuda(), T32.astype(np.float64)
    bits = synth.bf16_bits(T32)
    t = torch.from_numpy(bits.view(np.int16)).cuda().view(torch.bfloat16)
    return t, synth.bf16_to_f32(bits).astype(np.float64)


def to_np(t):
    return t.detach().cpu().double().numpy()



def check_trajectory(fhat, restart, ref, iters, normT2) -> int:
    """Compare a device run's F-hat and restart decisions with the oracle's (`ref`, an
    oracle.her_solve result) while F-hat moves by more than twice the tolerance; returns
    the number of iterations compared. F-hat = ||T||^2 / 2 - <P, A> + <G, A^T A> / 2 is a
    small difference of terms of size ||T||^2, so float32 rounding of the MTTKRP alone moves
    it by about u ||T||^2 (u = 2^-24): the tolerance is 1e-4 |F-hat| + 8 u ||T||^2."""
    prev = ref.fhat0
    checked = 0
    for k in range(iters):
        tol = 1e-4 * abs(ref.fhat[k]) + 2.0 ** -21 * normT2
        if abs(ref.fhat[k] - prev) < 2 * tol:
            break
        assert bool(restart[k]) == ref.restart[k], k
        assert abs(fhat[k] - ref.fhat[k]) <= tol, (k, fhat[k], ref.fhat[k], tol)
        prev = ref.fhat[k]
        checked += 1
    return checked
