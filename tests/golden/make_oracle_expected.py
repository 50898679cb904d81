"""Write the FP64 oracle's expected values for the full-size parity tests.

The oracle takes minutes per solve at the 128x128 workload, too long to run inside a
GPU test, so its results are computed once here, on the host, and stored next to this
script.  Only the oracle (``oracle/``) and the seeded input generators
(``paper_2410_09663_amd/workloads.py``, which hold none of the method's arithmetic)
are called.  Every file also stores a SHA-256 digest of the inputs it was computed
from; the tests recompute it from the generators and refuse a stale file.

Cases:
  c3_solve    one solve of the 128x128 workload (l = 32, CNN 2-32-32-32-1 GELU,
              N = 256, H = 10), explicit noise from the seeded host generator
              (seed 31), U_prev = 0: the smoothed means U_hat and X_hat of every slice.
  c2_loop     the 64x64 workload (l = 8, CNN 2-16-16-1 tanh, N = 128, H = 10) run as a
              20-step receding-horizon closed loop (Algorithm 1, lines 3-16) with the
              Philox noise stream keyed by 1000 + k at step k, the plant being the
              surrogate itself: the realised states, the applied controls and the
              closed-loop tracking cost.
  c3_loop     the 128x128 workload as a 4-step closed loop, the same way (keys 1000 + k).

Usage: python tests/golden/make_oracle_expected.py [case ...]   (default: every case)
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import cost as ocost  # noqa: E402
from oracle import enks, philox  # noqa: E402
from paper_2410_09663_amd import workloads as wl  # noqa: E402

C3_SOLVE_NOISE_SEED = 31
LOOP_STEPS = {"c2_loop": ("C2", 20), "c3_loop": ("C3", 4)}


def digest(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        a = np.ascontiguousarray(a)
        h.update(str(a.dtype).encode() + str(a.shape).encode())
        h.update(a.tobytes())
    return h.hexdigest()


def problem_digest(prob, extra=()) -> str:
    return digest(prob.B, *prob.weights, prob.X0, prob.Q, prob.R, *extra)


def c3_solve_inputs():
    p = wl.PRESETS["C3"]
    prob = wl.make_problem(p)
    Xref = wl.reference_window(p, 0)
    z = wl.host_noise(p.n, p.m, p.l, p.N, p.H, seed=C3_SOLVE_NOISE_SEED)
    return p, prob, Xref, z


def c3_solve_digest(prob, Xref, z) -> str:
    return problem_digest(prob, (Xref, z.Z_init, z.Z_W, z.Z_VX, z.Z_VU))


def loop_inputs(case):
    name, steps = LOOP_STEPS[case]
    p = wl.PRESETS[name]
    prob = wl.make_problem(p)
    refs = np.stack([wl.reference_at(p, k) for k in range(steps + p.H + 1)])
    return p, prob, steps, refs


def loop_digest(prob, refs, p) -> str:
    # the noise of the first step stands for the generator (its known-answer pins hold
    # the rest of the stream)
    z0 = philox.solve_noise(p.noise_seed_base, p.n, p.m, p.l, p.N, p.H)
    return problem_digest(prob, (refs,) + tuple(z0))


def make_c3_solve():
    p, prob, Xref, z = c3_solve_inputs()
    res = enks.solve(prob.B, prob.weights, p.activation, prob.X0, Xref, prob.Q, prob.Q, prob.R,
                     p.N, p.H, z.Z_init, z.Z_W, z.Z_VX, z.Z_VU)
    np.savez_compressed(os.path.join(HERE, "c3_solve_oracle.npz"),
                        U_mean=res.U_mean.astype(np.float32), X_mean=res.X_mean.astype(np.float32),
                        digest=np.array(c3_solve_digest(prob, Xref, z)))


def make_loop(case):
    p, prob, steps, refs = loop_inputs(case)
    Xs, Us = enks.closed_loop(prob.B, prob.weights, p.activation, prob.X0,
                              lambda k: refs[k:k + p.H + 1], prob.Q, prob.Q, prob.R, p.N, p.H, steps,
                              lambda k: philox.solve_noise(p.noise_seed_base + k, p.n, p.m, p.l,
                                                           p.N, p.H))
    cost = ocost.closed_loop_cost(Xs, Us, np.zeros((p.l, p.m)), refs[:steps + 1],
                                  prob.R.astype(np.float64), prob.Q.astype(np.float64))
    np.savez_compressed(os.path.join(HERE, f"{case}_oracle.npz"), Xs=Xs.astype(np.float32),
                        Us=Us.astype(np.float32), cost=np.array(cost),
                        digest=np.array(loop_digest(prob, refs, p)))


def main(cases):
    for c in cases:
        t0 = time.perf_counter()
        if c == "c3_solve":
            make_c3_solve()
        elif c in LOOP_STEPS:
            make_loop(c)
        else:
            raise SystemExit(f"unknown case {c}")
        print(f"{c}: {time.perf_counter() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["c3_solve", "c2_loop", "c3_loop"])
