"""Writes config1_bb72_p005.txt: the [[72,12,6]] workload decoded by the
double-precision CPU oracle alone (code capacity, i.i.d. bit flips p = 0.05,
10^4 seeded shots, min-sum alpha = 0.625, 100 first-BP iterations, |Phi| = 4
giving 16 trials of 20 iterations, lightest successful trial kept).

Calls only the oracle and the input generators; run from the repository root:
    python tests/golden/make_config1_record.py
"""
from __future__ import annotations

import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle.oracle import OracleLib, Params  # noqa: E402
from workloads import codes, gf2, shots  # noqa: E402

OUT = os.path.join(HERE, "config1_bb72_p005.txt")
P, N_SHOTS = 0.05, 10_000
Z95 = 1.959963984540054


def record() -> dict:
    code = codes.bb72()
    # the stream of the double-precision GPU test of this workload
    err, syn = shots.make_shots(code.hx, P, N_SHOTS, shots.stream_key(shots.MASTER_SEED, 531, code.n, 5000))
    prm = Params(max_iter=100, cand_max_iter=20, k=4, alpha=0.625)
    o = OracleLib().bpsf_batch(code.hx, syn, P, prm, prec="f64", threads=8)
    lx = gf2.logical_basis(code.hx, code.hz)
    resid = (err ^ o["correction"]).astype(np.int64)
    fail = (o["converged"] == 0) | ((resid @ lx.T.astype(np.int64)) & 1).any(axis=1)
    k, n = int(fail.sum()), N_SHOTS
    ph = k / n
    den = 1 + Z95 * Z95 / n
    cen = (ph + Z95 * Z95 / (2 * n)) / den
    half = Z95 * np.sqrt(ph * (1 - ph) / n + Z95 * Z95 / (4 * n * n)) / den
    return {"shots": n, "failed_first_bp": int(((o["winner"] >= 0) | (o["converged"] == 0)).sum()),
            "converged": int(o["converged"].sum()), "trial_winners": int((o["winner"] >= 0).sum()),
            "logical_failures": k, "ler": float(ph), "wilson95_lo": float(cen - half), "wilson95_hi": float(cen + half),
            "main_iterations": int(o["main_iterations"].sum()), "trial_iterations": int(o["trial_iterations"].sum())}


def main():
    r = record()
    with open(OUT, "w") as f:
        f.write("# [[72,12,6]] (l = m = 6, A = x^3 + y + y^2, B = y^3 + x + x^2), H_X 36 x 72, code capacity p = 0.05,\n"
                "# 10^4 seeded shots; double-precision oracle: alpha 0.625, 100 first-BP iterations, |Phi| = 4\n"
                "# (16 trials of 20 iterations), lightest successful trial. Written by make_config1_record.py.\n")
        for key, val in r.items():
            f.write(f"{key} {val!r}\n")
    print(open(OUT).read())


if __name__ == "__main__":
    main()
