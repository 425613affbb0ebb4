"""Writes the stored oracle values that the full-size GPU parity tests compare
against.  Calls only the oracle and the seeded input generators.

  periodic_2e6_ewald.npz   Gaussian-Ewald sum (oracle.ewald, truncation
                           e^-30, about 1e-13 relative) at 2,000 sampled
                           targets of the 2e6-point periodic workload
  clusters_4e6_direct.npz  direct FP64 sum (oracle.direct) at 10,000 sampled
                           targets of the 4e6-point clustered workload
  periodic_2e6_stresslet_ewald.npz
                           periodic stresslet sum (oracle.ewald.stresslet_ewald,
                           k = 0 term included) at 1,000 sampled targets of the
                           2e6-point periodic workload, with the seeded random
                           unit vectors of workloads.normals as n

Each file holds `idx` (target indices) and `u` (velocities, (m,3)).  Run from
the repository root:  python tests/golden/make_references.py [name ...]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402
from oracle.ewald import ewald, stresslet_ewald  # noqa: E402

REFS = {
    "periodic_2e6_ewald": ("periodic_2e6", 2000),
    "clusters_4e6_direct": ("clusters_4e6", 10000),
    "periodic_2e6_stresslet_ewald": ("periodic_2e6", 1000),
}


def make(name):
    cfg_name, m = REFS[name]
    cfg = workloads.CONFIGS[cfg_name]
    x, f = workloads.config(cfg_name)
    idx = workloads.sample_targets(x.shape[0], m, cfg["seed"])
    t0 = time.time()
    if name.endswith("stresslet_ewald"):
        u = stresslet_ewald(x, f, workloads.normals(x, cfg["seed"]), idx, E=30.0)
    elif cfg["periodic"]:
        u = ewald(x, f, idx, E=30.0)
    else:
        u = oracle.direct(x, f, idx)
    np.savez(os.path.join(HERE, name + ".npz"), idx=idx, u=u)
    print(f"{name}: {idx.size} targets, {time.time() - t0:.1f} s", flush=True)


if __name__ == "__main__":
    for name in sys.argv[1:] or list(REFS):
        make(name)
