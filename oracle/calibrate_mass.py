"""Write inputs/workloads.json: the seeded workloads and their calibrated masses.

The mass shift m is chosen as in Sec. 2.2 of the paper (eq. etamin): the
spectrum of D = D_0 + m I is that of D_0 moved by m, so with lambda* the
eigenvalue of the massless operator D_0 of smallest real part, m = t - Re
lambda* puts the eigenvalue closest to the imaginary axis at real part t.
lambda* is taken among the eigenvalues of D_0 nearest the origin, found by
shift-invert Arnoldi (SciPy ARPACK) on the oracle's sparse D_0.  The achieved
min |eig(D)| over those eigenvalues is stored beside m.

Run:  python -m oracle.calibrate_mass [names...]
Only the oracle (for D_0) and the seeded input generators are used.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

_HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(_HERE))

import inputs  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(_HERE), "inputs", "workloads.json")

# lattice, gauge recipe, target of min |eig(D)| and seeds
WORKLOADS = {
    "c1_32_b3": dict(N=32, beta=3.0, sweeps=200, gauge_seed=1, target=1e-2, rhs_seed=101, tv_seed=201,
                     n_levels=2, nrhs=1),
    "c2_128_b6": dict(N=128, beta=6.0, sweeps=500, gauge_seed=2, target=1e-3, rhs_seed=102, tv_seed=202,
                      n_levels=3, nrhs=1),
    "c3_256_b10": dict(N=256, beta=10.0, sweeps=500, gauge_seed=3, target=1e-4, rhs_seed=103, tv_seed=203,
                       n_levels=0, nrhs=1),
    "c4_512_b10": dict(N=512, beta=10.0, sweeps=500, gauge_seed=4, target=1e-4, rhs_seed=1001, tv_seed=204,
                       n_levels=0, nrhs=64),
    # the fourth field of the serving mix (with c2, c3 and c4)
    "s1_64_b3": dict(N=64, beta=3.0, sweeps=200, gauge_seed=5, target=1e-3, rhs_seed=105, tv_seed=205,
                     n_levels=0, nrhs=1),
}


def calibrate(w: dict, k: int = 12) -> dict:
    U = inputs.gauge_metropolis(w["N"], w["beta"], w["sweeps"], w["gauge_seed"])
    ptr, col, val = oracle.wilson_csr(U, 0.0)
    n = 2 * w["N"] ** 2
    D0 = sp.csc_matrix(sp.csr_matrix((val, col, ptr), shape=(n, n)))
    lam = spla.eigs(D0, k=k, sigma=0.0, which="LM", return_eigenvectors=False, tol=1e-12)
    i = int(np.argmin(lam.real))
    m = float(w["target"] - lam[i].real)
    achieved = float(np.min(np.abs(lam + m)))
    return dict(m=m, min_re_eig_D0=float(lam[i].real), min_abs_eig_D=achieved,
                eig_D0_near_0=[[float(z.real), float(z.imag)] for z in sorted(lam, key=lambda z: z.real)])


def main(names):
    data = {"workloads": {}}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    for name in names or WORKLOADS:
        w = dict(WORKLOADS[name])
        t0 = time.time()
        w.update(calibrate(w))
        print(f"{name}: m = {w['m']:.12g}, min|eig D| = {w['min_abs_eig_D']:.3e} ({time.time()-t0:.1f}s)",
              flush=True)
        data["workloads"][name] = w
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:])
