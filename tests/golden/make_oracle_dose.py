"""Writes the oracle's high-statistics reference doses for the dose parity
tests.  Calls only the oracle and the seeded input generators.

    python tests/golden/make_oracle_dose.py tiny 400000000 6 50
    python tests/golden/make_oracle_dose.py clinical10 200000000 8 50
    python tests/golden/make_oracle_dose.py hetero 300000000 8 50
    python tests/golden/make_oracle_dose.py hetero_lung 300000000 8 50

Arguments: workload, histories, threads (0 = all), batches.

tiny        60^3 water, 10x10 cm field aimed at the surface, SSD 100 cm,
            FP64 tally: tests/golden/oracle_dose_tiny.npz, dense float32
            dose and batch standard error (Gy per phase-space particle).
clinical10  the clinical-scale PSL workload: 1e7-particle phase space, 2 x 32
            log energy bins x 22 x 22 position bins of 5 mm, 10x10 cm open
            field with ROI culling and the jaw model, 128^3 water at 2.5 mm.
hetero      the heterogeneous workload at 2 mm: 256x256x160 phantom (water,
            lung ellipsoids, bone slabs), the random jaws and 40x40 fluence
            map of its seed.
hetero_lung the same phantom and fluence map, jaws X [0, 8], Y [-6, 6] cm
            at the SAD plane, placed so that the beam crosses both the lung
            ellipsoid and the bone slabs.

The three large workloads are stored sparsely: the voxels whose oracle dose
is at least 5% of its maximum (a bit mask over the volume), with dose and
standard error quantised to uint16 in units of max/65535 (dose) and
max/2^20 (standard error).  The quantisation step is below 1e-5 of the
maximum dose, three orders of magnitude under the standard errors it sits
beside.
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

HERE = os.path.dirname(os.path.abspath(__file__))
SIGMA_UNITS = 2.0 ** 20     # standard error in units of max / 2^20
SPARSE_FRACTION = 0.05


def hetero_lung_workload():
    """The heterogeneous workload's phantom and fluence map with jaws placed
    over the lung ellipsoid (X [0, 8], Y [-6, 6] cm at the SAD plane)."""
    import dataclasses
    wl = S.workload_heterogeneous()
    f = wl.fields[0]
    f2 = S.Field(0.0, 8.0, -6.0, 6.0, fluence=f.fluence)
    return dataclasses.replace(wl, name="heterogeneous-256x256x160-lung",
                               fields=[f2])


WORKLOADS = {
    "tiny": S.workload_tiny,
    "clinical10": lambda: S.workload_clinical(side=10.0),
    "hetero": S.workload_heterogeneous,
    "hetero_lung": hetero_lung_workload,
}


def store_sparse(path, dose, sigma, shape, **meta):
    mx = float(dose.max())
    keep = dose >= SPARSE_FRACTION * mx
    q = np.rint(dose[keep] / mx * 65535.0)
    qs = np.rint(sigma[keep] / mx * SIGMA_UNITS)
    if qs.max() > 65535:
        raise SystemExit("standard error too large for the uint16 scale")
    np.savez_compressed(path, shape=np.array(shape, np.int64),
                        dose_max=mx, mask=np.packbits(keep),
                        dose_q=q.astype(np.uint16),
                        sigma_q=qs.astype(np.uint16),
                        sparse_fraction=SPARSE_FRACTION, **meta)


def load_sparse(path):
    """(dose, sigma, mask) as dense float64 arrays [nz, ny, nx]; voxels not
    stored are NaN in dose and sigma."""
    z = np.load(path)
    shape = tuple(int(v) for v in z["shape"])
    n = int(np.prod(shape))
    keep = np.unpackbits(z["mask"])[:n].astype(bool)
    mx = float(z["dose_max"])
    dose = np.full(n, np.nan)
    sigma = np.full(n, np.nan)
    dose[keep] = z["dose_q"].astype(np.float64) * (mx / 65535.0)
    sigma[keep] = z["sigma_q"].astype(np.float64) * (mx / SIGMA_UNITS)
    return dose.reshape(shape), sigma.reshape(shape), keep.reshape(shape)


def main():
    which = sys.argv[1] if len(sys.argv) > 1 else "tiny"
    hist = int(float(sys.argv[2])) if len(sys.argv) > 2 else 400_000_000
    threads = int(sys.argv[3]) if len(sys.argv) > 3 else 0
    batches = int(sys.argv[4]) if len(sys.argv) > 4 else 50
    if which not in WORKLOADS:
        raise SystemExit("unknown workload " + which)
    wl = WORKLOADS[which]()
    oracle.build(force=False)
    t0 = time.time()
    dose, sigma, info = oracle.run_dose(wl, n_threads=threads,
                                        histories=hist, batches=batches)
    dt = time.time() - t0
    out = os.path.join(HERE, "oracle_dose_%s.npz" % which)
    meta = dict(histories=info["histories"], accepted=info["accepted"],
                seconds=dt, batches=batches, workload=wl.name)
    if which == "tiny":
        np.savez_compressed(out, dose=dose.astype(np.float32),
                            sigma=sigma.astype(np.float32), **meta)
    else:
        store_sparse(out, dose, sigma, wl.phantom.density.shape, **meta)
    print("wrote", out, info, "%.1f s" % dt)


if __name__ == "__main__":
    main()
