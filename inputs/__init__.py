"""Seeded synthetic inputs shared by the oracle-side tests and the GPU path.

This module holds no arithmetic of the solver: it only draws random numbers
and produces the problem data (gauge fields, right-hand sides, initial test
vectors) that both implementations receive as inputs.

* Gauge fields: quenched compact U(1) links from a Metropolis chain of the
  Wilson plaquette action (Sec. 2, eq. wilsongauge).  The weight is
  exp(+beta * sum_p cos(theta_p)); the paper prints the action without the
  customary "1 -" but states that beta -> infinity drives the links to one,
  which fixes the sign.  Hot start (theta uniform in [-pi, pi)), four link
  classes per sweep (x-links on even base sites, x-links on odd base sites,
  then y-links even / odd; links of one class share no plaquette), one hit per
  link with proposal theta + delta*(2u - 1), delta = min(pi, 2/sqrt(beta)).
* Right-hand sides and initial test vectors: complex Gaussians with real and
  imaginary parts i.i.d. N(0, 1/2), i.e. variance one (Sec. 4).

Field layouts (interleaved complex128):
  gauge  U[mu][y][x]          mu = 0: link (x,y)->(x+1,y); mu = 1: (x,y)->(x,y+1)
  spinor psi[y][x][s]         full lattice, 2 spin components
  reduced v[y][xh][s]         even sites only, x = 2*xh + (y mod 2)
"""
from __future__ import annotations

import json
import os

import numpy as np

__all__ = [
    "gauge_metropolis", "gauge_random", "gauge_free", "gaussian", "workload",
    "workload_names", "load_gauge",
]

_HERE = os.path.dirname(os.path.abspath(__file__))


def gauge_free(N: int) -> np.ndarray:
    """Unit links (the free field of Sec. 2)."""
    return np.ones((2, N, N), dtype=np.complex128)


def gauge_random(N: int, seed: int) -> np.ndarray:
    """Links with independent uniform phases (the beta -> 0 limit)."""
    rng = np.random.default_rng(seed)
    return np.exp(1j * rng.uniform(-np.pi, np.pi, size=(2, N, N)))


def _metropolis_theta(N: int, beta: float, sweeps: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    th = rng.uniform(-np.pi, np.pi, size=(2, N, N))  # th[mu, y, x]
    delta = min(np.pi, 2.0 / np.sqrt(beta)) if beta > 0 else np.pi
    yy, xx = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    parity = (xx + yy) % 2

    def sh(a, dx, dy):
        # value at (x+dx, y+dy)
        return np.roll(np.roll(a, -dx, axis=1), -dy, axis=0)

    for _ in range(sweeps):
        for mu in (0, 1):
            for par in (0, 1):
                tx, ty = th[0], th[1]
                if mu == 0:
                    # plaquette at z:     +th + [ty(z+x) - tx(z+y) - ty(z)]
                    # plaquette at z-y:   -th + [tx(z-y) + ty(z-y+x) - ty(z-y)]
                    a = sh(ty, 1, 0) - sh(tx, 0, 1) - ty
                    b = sh(tx, 0, -1) + sh(ty, 1, -1) - sh(ty, 0, -1)
                    old = tx
                    loc = lambda t: np.cos(t + a) + np.cos(b - t)
                else:
                    # plaquette at z:     -th + [tx(z) + ty(z+x) - tx(z+y)]
                    # plaquette at z-x:   +th + [tx(z-x) - tx(z-x+y) - ty(z-x)]
                    a = tx + sh(ty, 1, 0) - sh(tx, 0, 1)
                    b = sh(tx, -1, 0) - sh(tx, -1, 1) - sh(ty, -1, 0)
                    old = ty
                    loc = lambda t: np.cos(a - t) + np.cos(t + b)
                prop = old + delta * (2.0 * rng.random((N, N)) - 1.0)
                dS = beta * (loc(prop) - loc(old))
                acc = (rng.random((N, N)) < np.exp(np.minimum(dS, 0.0))) & (parity == par)
                new = np.where(acc, prop, old)
                new = np.mod(new + np.pi, 2.0 * np.pi) - np.pi
                th[mu] = new
    return th


def gauge_metropolis(N: int, beta: float, sweeps: int, seed: int) -> np.ndarray:
    """U(1) links exp(i theta) after `sweeps` Metropolis sweeps (shape (2, N, N))."""
    return np.exp(1j * _metropolis_theta(N, beta, sweeps, seed))


def plaquette_cos(U: np.ndarray) -> np.ndarray:
    """cos(theta_p) of every plaquette (used to check the gauge generator)."""
    tx, ty = np.angle(U[0]), np.angle(U[1])
    sh = lambda a, dx, dy: np.roll(np.roll(a, -dx, axis=1), -dy, axis=0)
    return np.cos(tx + sh(ty, 1, 0) - sh(tx, 0, 1) - ty)


def gaussian(shape, seed: int) -> np.ndarray:
    """Complex Gaussian array, real and imaginary parts i.i.d. N(0, 1/2)."""
    rng = np.random.default_rng(seed)
    shape = tuple(np.atleast_1d(shape))
    z = rng.standard_normal(shape + (2,)) * np.sqrt(0.5)
    return z[..., 0] + 1j * z[..., 1]


def _workloads():
    with open(os.path.join(_HERE, "workloads.json")) as f:
        return json.load(f)


def workload_names():
    return list(_workloads()["workloads"].keys())


def workload(name: str) -> dict:
    """Workload record: lattice, gauge recipe and seed, calibrated mass, seeds."""
    w = dict(_workloads()["workloads"][name])
    w["name"] = name
    return w


_GAUGE_CACHE: dict = {}


def load_gauge(w: dict) -> np.ndarray:
    """Gauge field of a workload record (generated from its seed; memoised)."""
    key = (w["N"], w["beta"], w["sweeps"], w["gauge_seed"])
    if key not in _GAUGE_CACHE:
        _GAUGE_CACHE[key] = gauge_metropolis(w["N"], w["beta"], w["sweeps"], w["gauge_seed"])
    return _GAUGE_CACHE[key]
