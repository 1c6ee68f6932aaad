"""Write tests/golden/oracle_fits.json: the FP64 oracle's final fit on named workloads.

    python tests/golden/make_golden.py cube50_r10 cube400_r32_corr quad128_r64_sparse:bf16:20
    python tests/golden/make_golden.py batch256:200
    python tests/golden/make_golden.py tucker_video_r10

Calls only the oracle (and the seeded input generator for its inputs). The oracle sees
the float32 values of the tensor and the initial factors, as the GPU does; a spec
`name:bf16` rounds the tensor to bfloat16 first (round to nearest even, as the inputs of
the GPU tests are rounded),
for workloads whose tensor is stored in that format, and a third field `:K` overrides the
workload's outer-iteration count. For each spec it records the final relative error / fit
of Algorithm 2 (HER with A-HALS, the paper's default parameters; the fit is taken against
the tensor the oracle solved), the number of restarts, and the F-hat trace, under the key
`name` (float32 tensor, the workload's own count) or the spec itself. `batch256:K` records
the fits after K iterations of 16 problems of the 256-problem batch (see `batch_pick`); a
Tucker-format workload name records Algorithm 2 on the format (Appendix A).
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(HERE, "oracle_fits.json")


def run(spec: str) -> dict:
    parts = spec.split(":")
    name = parts[0]
    dtype = parts[1] if len(parts) > 1 else "f32"
    w = synth.WORKLOADS[name]
    iters = int(parts[2]) if len(parts) > 2 else w["iters"]
    pr = synth.workload(name)
    T32 = pr.T.astype(np.float32)
    if dtype == "bf16":
        T64 = synth.bf16_to_f32(synth.bf16_bits(T32)).astype(np.float64)
    elif dtype == "f32":
        T64 = T32.astype(np.float64)
    else:
        raise ValueError(f"unknown tensor format {dtype}")
    del T32
    A0 = [a.astype(np.float32).astype(np.float64) for a in pr.A0]
    del pr
    t0 = time.perf_counter()
    res = oracle.her_solve(T64, A0, iters)
    dt = time.perf_counter() - t0
    rel = oracle.relative_error(T64, res.factors)
    return dict(workload=name, tensor=dtype, iters=iters, relerr=rel, fit=1.0 - rel,
                restarts=int(sum(res.restart)), fhat=res.fhat, fhat0=res.fhat0,
                oracle_seconds=dt, cpu_count=os.cpu_count())


def batch_pick(specs):
    """The 16 problems of the 256-problem batch that the GPU test checks: the five largest by
    cost (I_1 I_2 I_3 r), the smallest, and one from each tenth of the cost order."""
    cost = [np.prod(s[:3]) * s[3] for s in specs]
    order = [int(i) for i in np.argsort(cost, kind="stable")]
    pick = list(dict.fromkeys(order[-5:] + [order[0]] +
                              [order[(k * len(order)) // 10] for k in range(1, 10)] +
                              [order[len(order) // 20]]))
    return pick[:16]


def run_batch(iters: int) -> dict:
    """Oracle fits of the picked batch problems after `iters` outer iterations."""
    specs = synth.batch_specs(256)
    out = {"iters": iters, "fits": {}}
    t0 = time.perf_counter()
    for b in batch_pick(specs):
        pr = synth.batch_problem(specs[b], b)
        T64 = pr.T.astype(np.float32).astype(np.float64)
        A0 = [a.astype(np.float32).astype(np.float64) for a in pr.A0]
        res = oracle.her_solve(T64, A0, iters)
        out["fits"][str(b)] = oracle.fit(T64, res.factors)
        print(f"  batch problem {b} {specs[b]}: fit {out['fits'][str(b)]:.8f}", flush=True)
    out["oracle_seconds"] = time.perf_counter() - t0
    return out


def run_tucker(name: str) -> dict:
    """Algorithm 2 on a Tucker-format workload (Appendix A) from the float32 core, bases and
    initial factors the GPU receives; the fit by the format's own residual norm."""
    w = synth.TUCKER_WORKLOADS[name]
    pr = synth.tucker_workload(name)
    core = pr.core.astype(np.float32).astype(np.float64)
    bases = [U.astype(np.float32).astype(np.float64) for U in pr.bases]
    A0 = [a.astype(np.float32).astype(np.float64) for a in pr.A0]
    t0 = time.perf_counter()
    res = oracle.tucker_her_solve(core, bases, A0, w["iters"])
    dt = time.perf_counter() - t0
    rel = oracle.tucker_relative_error(core, bases, res.factors)
    return dict(workload=name, tensor="tucker_f32", iters=w["iters"], relerr=rel, fit=1.0 - rel,
                restarts=int(sum(res.restart)), fhat=res.fhat, fhat0=res.fhat0,
                oracle_seconds=dt, cpu_count=os.cpu_count())


def main(names):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for n in names:
        print(f"running {n} ...", flush=True)
        if n in synth.TUCKER_WORKLOADS:
            data[n] = run_tucker(n)
            print(f"{n}: fit {data[n]['fit']:.8f} in {data[n]['oracle_seconds']:.1f}s",
                  flush=True)
            json.dump(data, open(OUT, "w"), indent=1)
            continue
        if n.startswith("batch256"):
            data[n] = run_batch(int(n.split(":")[1]))
            json.dump(data, open(OUT, "w"), indent=1)
            continue
        data[n] = run(n)
        print(f"{n}: fit {data[n]['fit']:.8f} in {data[n]['oracle_seconds']:.1f}s", flush=True)
        json.dump(data, open(OUT, "w"), indent=1)


if __name__ == "__main__":
    main(sys.argv[1:])
