"""Seeded synthetic inputs shared by the tests, the smoke check and the
benchmark.

This module holds problem descriptions and random draws only -- none of the
method's arithmetic.  Both the GPU library and the oracle derive everything
else (rest weights, relaxation rates, equilibria) on their own.

Workloads (all lid-driven cavities unless noted; lattice units dx = dt = 1):

  CAVITY_64x32_F64       64 x 32, r = 2, Re = 100, U = 0.05, gamma = 1, FP64
  CAVITY_1024x512_F32    1024 x 512, r = 2, Re = 1000, U = 0.05, gamma = 0.1,
                         FP32, residual check every 1000 steps, tol 1e-8
  CAVITY_4096x2048_16B   4096 x 2048, r = 0.5, Re = 2000, U = 0.05,
                         gamma = 0.05, FP16 / BF16 deviation storage
  *_MA006 / *_MA002      the same grids with the lid at Ma = 0.06 / 0.02,
                         inside the scheme's stable range
  BATCH_256              256 instances drawn with numpy seed 0
  SERVE_POISSON          Poisson request trace drawn with numpy seed 1
"""
from __future__ import annotations

import math
from dataclasses import asdict, dataclass

import numpy as np


@dataclass(frozen=True)
class Cavity:
    name: str
    nx: int
    ny: int
    r: float
    re: float
    u_lid: float
    gamma: float
    storage: str          # "f64" | "f32" | "f16" | "bf16"
    check_every: int = 1000
    tol: float = 1e-8
    max_steps: int = 20000

    def dict(self):
        return asdict(self)


CAVITY_64x32_F64 = Cavity("cavity_64x32_r2_re100_g1_f64", 64, 32, 2.0, 100.0, 0.05, 1.0, "f64",
                          check_every=1000, tol=1e-8, max_steps=20000)
CAVITY_1024x512_F32 = Cavity("cavity_1024x512_r2_re1000_g0.1_f32", 1024, 512, 2.0, 1000.0, 0.05,
                             0.1, "f32", check_every=1000, tol=1e-8, max_steps=10 ** 9)
CAVITY_4096x2048_F16 = Cavity("cavity_4096x2048_r0.5_re2000_g0.05_f16", 4096, 2048, 0.5, 2000.0,
                              0.05, 0.05, "f16", check_every=1000, tol=1e-8, max_steps=10 ** 9)
CAVITY_4096x2048_BF16 = Cavity("cavity_4096x2048_r0.5_re2000_g0.05_bf16", 4096, 2048, 0.5,
                               2000.0, 0.05, 0.05, "bf16", check_every=1000, tol=1e-8,
                               max_steps=10 ** 9)
# the same grid with FP32 storage: HBM-resident (604 MB) roofline case
CAVITY_4096x2048_F32 = Cavity("cavity_4096x2048_r0.5_re2000_g0.05_f32", 4096, 2048, 0.5, 2000.0,
                              0.05, 0.05, "f32", check_every=1000, tol=1e-8, max_steps=10 ** 9)


def deviation_noise(nx: int, ny: int, seed: int, amplitude: float) -> np.ndarray:
    """Uniform random numbers in [-amplitude, amplitude], shape [9][ny][nx]
    (float64): a perturbation that each side adds to its own rest state."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-amplitude, amplitude, size=(9, ny, nx))


@dataclass(frozen=True)
class Instance:
    nx: int
    ny: int
    r: float
    gamma: float
    re: float
    u_lid: float = 0.05


def batch_instances(n: int = 256, seed: int = 0) -> list[Instance]:
    """Uneven cavity instances: Nx, Ny log-uniform in [64, 512], r uniform in
    {0.5, 1, 2, 4}, gamma uniform in [0.05, 1], Re log-uniform in [100, 5000],
    lid 0.05 -- drawn in that order per instance."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        nx = int(round(math.exp(rng.uniform(math.log(64), math.log(512)))))
        ny = int(round(math.exp(rng.uniform(math.log(64), math.log(512)))))
        r = float(rng.choice([0.5, 1.0, 2.0, 4.0]))
        gamma = float(rng.uniform(0.05, 1.0))
        re = float(math.exp(rng.uniform(math.log(100), math.log(5000))))
        out.append(Instance(nx, ny, r, gamma, re))
    return out


@dataclass(frozen=True)
class Request:
    arrival_s: float
    inst: Instance


def poisson_trace(n: int, rate_per_s: float, seed: int = 1) -> list[Request]:
    """Steady-state solve requests arriving as a Poisson process: Nx
    log-uniform in [128, 2048], Ny log-uniform in [128, 1024], r, gamma, Re as
    in batch_instances."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for _ in range(n):
        t += float(rng.exponential(1.0 / rate_per_s))
        nx = int(round(math.exp(rng.uniform(math.log(128), math.log(2048)))))
        ny = int(round(math.exp(rng.uniform(math.log(128), math.log(1024)))))
        r = float(rng.choice([0.5, 1.0, 2.0, 4.0]))
        gamma = float(rng.uniform(0.05, 1.0))
        re = float(math.exp(rng.uniform(math.log(100), math.log(5000))))
        out.append(Request(t, Instance(nx, ny, r, gamma, re)))
    return out

# Lid speed at Ma = U / c_s = 0.06 on a lattice with q = 1 (c_s = 1/sqrt(3)):
# the Mach number the paper runs its gamma = 0.1 and 0.08 cases at (Sec. 5.2).
MA006_LID = 0.06 / math.sqrt(3.0)

# 1024 x 512 cavity of CAVITY_1024x512_F32 with the lid at Ma = 0.06: the
# named lid speed 0.05 with gamma = 0.1 is outside the scheme's stable range
# (the FP64 oracle diverges within about 100 steps), this one is not.
CAVITY_1024x512_F32_MA006 = Cavity("cavity_1024x512_r2_re1000_g0.1_ma0.06_f32", 1024, 512, 2.0,
                                   1000.0, MA006_LID, 0.1, "f32", check_every=1000, tol=1e-8,
                                   max_steps=10 ** 9)

# The 4096 x 2048 shallow cavity (r = 0.5, Re = 2000, gamma = 0.05) with the
# named lid speed 0.05 is Ma = 0.17 on this lattice, far outside the scheme's
# stable range for gamma = 0.05 (the FP64 oracle blows up within 200 steps at
# 1/16 scale).  At full size Ma = 0.06 with gamma = 0.05 blows up as well
# (about step 2000, FP64 included); the paper itself pairs gamma = 0.05 with
# Ma = 0.02 (deep cavity, Sec. 5.2) and notes that the smallest stable gamma
# grows with the Mach number.  Companion: Ma = 0.02, U = 0.02 q / sqrt(3),
# stable over 30000 steps at full size in FP32 and FP16.
MA006_LID_R05 = 0.06 * 0.5 / math.sqrt(3.0)
MA002_LID_R05 = 0.02 * 0.5 / math.sqrt(3.0)
CAVITY_4096x2048_MA002 = {
    s: Cavity(f"cavity_4096x2048_r0.5_re2000_g0.05_ma0.02_{s}", 4096, 2048, 0.5, 2000.0,
              MA002_LID_R05, 0.05, s, check_every=1000, tol=1e-8, max_steps=10 ** 9)
    for s in ("f64", "f32", "f16", "bf16")
}
