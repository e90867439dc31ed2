"""Writes tests/golden/cfg2_full_E.npz: the FP64 oracle's signal for the
full two-phase axon workload (128^3, mirror faces, 6 oblique directions,
10^4 steps), every 10th step and the last.  Calls only the oracle and the
seeded inputs; run with `python tests/golden/make_cfg2_full.py [threads]`
(about an hour on 8 cores)."""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as w  # noqa: E402


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else 8
    cfg = w.make_config("cfg2")
    K = len(cfg["f"])
    keep = np.unique(np.concatenate([np.arange(0, K + 1, 10), [K]]))
    out = []
    for q in range(len(cfg["gG0"])):
        t0 = time.time()
        E, _ = oracle.simulate_config(cfg, q=[q], threads=threads)
        out.append(E[0][keep])
        print(f"q={q} done in {time.time() - t0:.0f} s", flush=True)
    np.savez_compressed(os.path.join(os.path.dirname(os.path.abspath(__file__)), "cfg2_full_E.npz"),
                        steps=keep, E=np.array(out), gG0=cfg["gG0"],
                        note="FP64 oracle, two-phase axon workload 128^3, seed 2")


if __name__ == "__main__":
    main()
