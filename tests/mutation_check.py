"""Mutation check of the oracle's pins (CPU only; not collected by pytest).

Each mutation plants one plausible mistake in a copy of the oracle (a dropped term, a
wrong sign, index or operand) and runs the CPU test suite on that copy; the check
passes when every mutation makes at least one test fail.  The repository itself is
never modified.

Usage: python tests/mutation_check.py [name ...]   (default: every mutation)
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (name, file, original text, mutated text)
MUTATIONS = [
    ("lag update dropped (only the newest slice analysed)", "oracle/enks.py",
     "traj[:, :j] = Xcal_upd.reshape(N, j, r, m)",
     "traj[:, t] = Xcal_upd.reshape(N, j, r, m)[:, t]"),
    ("innovation sign flipped", "oracle/enks.py",
     "Xcal_upd = Xcal + np.matmul(K, Ybar_t[None] - Y)",
     "Xcal_upd = Xcal - np.matmul(K, Ybar_t[None] - Y)"),
    ("Q_U and Q_dU swapped", "oracle/enks.py",
     "L_dU = _chol_lower(QdU)", "L_dU = _chol_lower(QU)"),
    ("gain with an untransposed factor", "oracle/enks.py",
     "K = np.linalg.solve(Ly.T, np.linalg.solve(Ly, Sxy.T)).T",
     "K = np.linalg.solve(Ly, np.linalg.solve(Ly, Sxy.T)).T"),
    # (the trajectory mean inside the analysis cancels: sum_i D^i = 0, so any constant
    # subtracted from every member leaves Sigma^{XY} unchanged; that mutant is equivalent)
    ("missing 1/N in the observation mean", "oracle/enks.py",
     "Ymean = Y.mean(axis=0)", "Ymean = Y.sum(axis=0)"),
    ("missing 1/N in the smoothed means", "oracle/enks.py",
     "mean = traj.mean(axis=0)", "mean = traj.sum(axis=0)"),
    ("observations taken from the previous slice", "oracle/enks.py",
     "Y = np.concatenate([traj[:, t, :n] + VX, traj[:, t, n:n + l] + VU], axis=1)",
     "Y = np.concatenate([traj[:, t - 1, :n] + VX, traj[:, t - 1, n:n + l] + VU], axis=1)"),
    ("no control spread in the initial ensemble", "oracle/enks.py",
     "traj[:, 0, n:n + l, :] = U_prev + W0", "traj[:, 0, n:n + l, :] = U_prev"),
    ("closed loop applies the second slice", "oracle/enks.py",
     "Uk = res.U_mean[0]", "Uk = res.U_mean[1]"),
    ("closed loop without the U_prev hand-over", "oracle/enks.py",
     "        Up = Uk\n", "        Up = Up\n"),
    ("conv taps flipped vertically (convolution, not cross-correlation)", "oracle/cnn.py",
     "pad[s:e, :, a:a + n, b_:b_ + m]", "pad[s:e, :, 2 - a:2 - a + n, b_:b_ + m]"),
    ("activation after the last layer", "oracle/cnn.py",
     "if ell < L - 1:", "if ell < L:"),
    ("tanh computed as GELU", "oracle/cnn.py",
     "return np.tanh(x)", "return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))"),
    ("control lift transposed", "oracle/cnn.py",
     "BU = np.matmul(B, U)", "BU = np.matmul(B, U[..., ::-1, :])"),
    ("cost increment with the wrong sign", "oracle/cost.py",
     "dU = Us[k] - Uprev", "dU = Us[k] + Uprev"),
    ("Philox multiplier mistyped", "oracle/philox.py",
     "M0 = 0xD2511F53", "M0 = 0xD2511F55"),
    ("Box-Muller sine branch", "oracle/philox.py", "np.cos(", "np.sin("),
    ("right transform without the Gram inverse", "oracle/transform.py",
     "np.linalg.solve(", "(lambda A, B: B)("),
]


def run(mutation) -> tuple:
    name, rel, old, new = mutation
    tmp = tempfile.mkdtemp(prefix="oic_mut_")
    try:
        for d in ("oracle", "tests", "paper_2410_09663_amd", "include"):
            shutil.copytree(os.path.join(ROOT, d), os.path.join(tmp, d),
                            ignore=shutil.ignore_patterns("__pycache__", "*.npz"))
        for f in ("pytest.ini", "bench.py", "__graft_entry__.py"):
            shutil.copy(os.path.join(ROOT, f), tmp)
        if rel:
            path = os.path.join(tmp, rel)
            with open(path) as f:
                src = f.read()
            if old not in src:
                return name, None, f"pattern not found in {rel}"
            with open(path, "w") as f:
                f.write(src.replace(old, new))
        res = subprocess.run([sys.executable, "-m", "pytest", "tests", "-m", "not gpu and not slow", "-x",
                              "-q", "-p", "no:cacheprovider"], cwd=tmp, capture_output=True, text=True)
        lines = res.stdout.splitlines()
        failed = [ln for ln in lines if ln.startswith("FAILED")]
        errors = [ln for ln in lines if ln.startswith("ERROR")]
        if errors:  # a suite that cannot even run catches nothing
            return name, None, errors[0]
        return name, bool(failed), failed[0] if failed else (lines[-1] if lines else "")
    finally:
        shutil.rmtree(tmp, ignore_errors=True)


def main(names):
    chosen = [m for m in MUTATIONS if not names or m[0] in names]
    _, failed, detail = run(("unmutated copy", None, None, None))
    if failed is not False:
        print(f"the unmutated copy does not pass: {detail}")
        return 1
    ok = True
    for m in chosen:
        name, caught, detail = run(m)
        status = {True: "caught", False: "MISSED", None: "BROKEN"}[caught]
        ok &= caught is True
        print(f"{status:7s} {name}: {detail}", flush=True)
    print("every mutation caught" if ok else "some mutations were not caught")
    return 0 if ok else 1


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
