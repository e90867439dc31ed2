"""Writes tests/golden/cfg2_64_full_E.npz: the FP64 oracle's signal for the
two-phase axon workload on a 64^3 lattice (same packing law, seed, spacing,
time step, waveform and mirror faces as the 128^3 workload), over the full
10^4 steps, for the q-samples 0, 3 and 4 (xy-, xz- and yz-oblique
directions), every 10th step and the last.  Calls only the oracle and the
seeded inputs; run with `python tests/golden/make_cfg2_full.py [threads]`
(about 40 minutes on 6 cores)."""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as w  # noqa: E402

N = 64
QS = (0, 3, 4)


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else 8
    cfg = w.make_config("cfg2", n=N)
    K = len(cfg["f"])
    keep = np.unique(np.concatenate([np.arange(0, K + 1, 10), [K]]))
    out = []
    for q in QS:
        t0 = time.time()
        E, _ = oracle.simulate_config(cfg, q=[q], threads=threads)
        out.append(E[0][keep])
        print(f"q={q} done in {time.time() - t0:.0f} s", flush=True)
    np.savez_compressed(os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                     "cfg2_64_full_E.npz"),
                        n=N, qs=np.array(QS), steps=keep, E=np.array(out),
                        gG0=cfg["gG0"][list(QS)])


if __name__ == "__main__":
    main()
