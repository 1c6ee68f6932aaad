"""Write tests/golden/oracle_fits.json: the FP64 oracle's final fit on named workloads.

    python tests/golden/make_golden.py cube50_r10 cube400_r32_corr ...

Calls only the oracle (and the seeded input generator for its inputs). The oracle sees
the float32 values of the tensor and the initial factors, as the GPU does. For each
workload it records the final relative error / fit of Algorithm 2 (HER with A-HALS,
the paper's default parameters) after the workload's outer-iteration count, the number
of restarts, and the F-hat trace.
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


def run(name: str) -> dict:
    w = synth.WORKLOADS[name]
    pr = synth.workload(name)
    T64 = pr.T.astype(np.float32).astype(np.float64)
    A0 = [a.astype(np.float32).astype(np.float64) for a in pr.A0]
    del pr
    t0 = time.perf_counter()
    res = oracle.her_solve(T64, A0, w["iters"])
    dt = time.perf_counter() - t0
    rel = oracle.relative_error(T64, res.factors)
    return dict(workload=name, iters=w["iters"], relerr=rel, fit=1.0 - rel,
                restarts=int(sum(res.restart)), fhat=res.fhat, fhat0=res.fhat0,
                oracle_seconds=dt, cpu_count=os.cpu_count())


def main(names):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for n in names:
        print(f"running {n} ...", flush=True)
        data[n] = run(n)
        print(f"{n}: fit {data[n]['fit']:.8f} in {data[n]['oracle_seconds']:.1f}s", flush=True)
        json.dump(data, open(OUT, "w"), indent=1)


if __name__ == "__main__":
    main(sys.argv[1:])
