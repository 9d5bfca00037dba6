"""Writes the oracle's high-statistics reference dose for the dose parity
tests.  Calls only the oracle and the seeded input generators.

    python tests/golden/make_oracle_dose.py tiny 400000000 6 50

writes tests/golden/oracle_dose_tiny.npz with the dose and its batch
standard error (Gy per phase-space particle, from 50 batches) of the 60^3
water workload (10x10 cm field aimed at the surface, SSD 100 cm), plus the
run metadata.
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(
    os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import psl_synth as S  # noqa: E402


def main():
    which = sys.argv[1] if len(sys.argv) > 1 else "tiny"
    hist = int(float(sys.argv[2])) if len(sys.argv) > 2 else 400_000_000
    threads = int(sys.argv[3]) if len(sys.argv) > 3 else 0
    batches = int(sys.argv[4]) if len(sys.argv) > 4 else 50
    if which != "tiny":
        raise SystemExit("unknown workload " + which)
    wl = S.workload_tiny()
    oracle.build(force=False)
    t0 = time.time()
    dose, sigma, info = oracle.run_dose(wl, n_threads=threads,
                                        histories=hist, batches=batches)
    dt = time.time() - t0
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                       "oracle_dose_%s.npz" % which)
    np.savez_compressed(out, dose=dose.astype(np.float32),
                        sigma=sigma.astype(np.float32),
                        histories=info["histories"],
                        accepted=info["accepted"], seconds=dt, batches=batches,
                        workload=wl.name)
    print("wrote", out, info, "%.1f s" % dt)


if __name__ == "__main__":
    main()
