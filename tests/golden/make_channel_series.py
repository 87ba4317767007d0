"""Writes tests/golden/channel_96x48x48_qstar.npz: the FP64 oracle's long-run
q* series of the 96 x 48 x 48 channel TO-LRS workload (12 QoIs,
Smagorinsky C_s = 0.1, LRS h = 0 active from step S0), and the series of its
twin started one unit in the last place away (the chaos floor of the KS
parity bar, Sec. 3.1, eq. KS).  Calls only the oracle and the seeded input
generators; run from the repository root:

    python tests/golden/make_channel_series.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

import oracle  # noqa: E402
import synth  # noqa: E402

STEPS, S0 = 3000, 500
GRID = (96, 48, 48)
OUT = os.path.join(ROOT, "tests", "golden", "channel_96x48x48_qstar.npz")


def case():
    """The workload of the test (shared with it)."""
    cfg, u0 = synth.channel_workload(*GRID)
    nb, dmin, dmax = synth.channel_bands(GRID[1])
    C, mu, S = synth.lrs_model_channel(12, 7, 9)
    cargs = dict(mode="lrs", spinup=S0, C=C, mu=mu, Sigma=S, seed=11, nbands=nb, dmin=dmin, dmax=dmax)
    return cfg, u0, synth.QOIS_3D, cargs


def twin_velocity(u0):
    return u0 * (1 + 2.2e-16 * np.random.default_rng(1).choice([-1, 1], size=u0.shape))


def run(u0):
    cfg, _, qois, cargs = case()
    o = oracle.Oracle(**cfg)
    o.init(u0)
    o.set_closure(oracle.make_closure(qois, **cargs))
    t = time.time()
    for k in range(STEPS // 100):
        o.step(100)
        print(f"  step {(k + 1) * 100} ({time.time() - t:.0f} s)", flush=True)
    return o.record_arrays()["q"][S0:]


def main():
    _, u0, _, _ = case()
    qo = run(u0)
    qt = run(twin_velocity(u0))
    np.savez_compressed(OUT, oracle=qo, twin=qt, steps=STEPS, s0=S0)
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()
