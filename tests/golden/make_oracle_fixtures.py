"""Write oracle results for the large workloads (run on the CPU; calls only
oracle/ and the seeded input generator).

  python tests/golden/make_oracle_fixtures.py [c3] [c5]

c3: n=20, 8 layers, CZ ladder, all 64 samples: expectation values, dL/dw over
    the batch, dL/dx per sample (the oracle's VJP, complex128).
c5: n=26, 10 layers, CNOT ring, the first 2 samples: the same quantities for
    that 2-sample batch (amplitude-parallel oracle).
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402


def make(name, batch, par_mode, threads):
    wl = W.config_workload(name, batch=batch)
    t0 = time.time()
    ev, gw, gx = oracle.vjp(wl.circuit, wl.inputs, wl.weights, wl.grad_out, threads=threads,
                            par_mode=par_mode)
    dt = time.time() - t0
    path = os.path.join(HERE, f"oracle_{name}_b{wl.batch}.npz")
    np.savez_compressed(path, expvals=ev, grad_w=gw, grad_x=gx, batch=wl.batch,
                        seconds=dt, threads=threads)
    print(f"{path}: {dt:.1f} s", flush=True)


if __name__ == "__main__":
    which = sys.argv[1:] or ["c3", "c5"]
    thr = os.cpu_count() or 1
    if "c3" in which:
        make("c3", None, 0, thr)
    if "c5" in which:
        make("c5", 2, 1, thr)
