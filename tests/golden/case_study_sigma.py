"""Writes case_study_gaussian.txt: the width of the case study's initial
Gaussian (Sec. 6.5: Heat-2D 5-point, 9600 x 9600, CFL number 0.23,
3.8e6 steps, peak 100 degC, centre cooling to 52.0 degC).

The paper gives neither the width nor the boundary temperature.  With the
zero rule (edges held at 0) and amplitude 100, the width sigma (in cells) is
chosen by bisection so that the closed-form solution (oracle.heat_spectral)
has 52.0 at the centre cells after 3.8e6 steps.  Only the oracle is called.

    python tests/golden/case_study_sigma.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402

N, MU, STEPS, AMP, TARGET = 9600, 0.23, 3_800_000, 100.0, 52.0


def centre(sigma):
    u = oracle.heat_spectral(synth.gaussian_plate(N, sigma, AMP), MU, STEPS)
    c = N // 2 - 1
    return float(u[c, c])


def main():
    lo, hi = 500.0, 4000.0  # centre(lo) < TARGET < centre(hi)
    flo, fhi = centre(lo), centre(hi)
    print(f"sigma {lo}: {flo:.4f}  sigma {hi}: {fhi:.4f}", flush=True)
    assert flo < TARGET < fhi
    for _ in range(14):
        mid = 0.5 * (lo + hi)
        f = centre(mid)
        print(f"sigma {mid:.3f}: centre {f:.6f}", flush=True)
        if f < TARGET:
            lo = mid
        else:
            hi = mid
    sigma = round(0.5 * (lo + hi), 1)
    f = centre(sigma)
    with open(os.path.join(HERE, "case_study_gaussian.txt"), "w") as fh:
        fh.write("# Case study initial field (Sec. 6.5): amplitude * exp(-r^2 / (2 sigma^2)) on 9600 x 9600,\n")
        fh.write("# centred at ((n-1)/2, (n-1)/2); sigma chosen so that the closed-form zero-rule solution\n")
        fh.write("# after 3.8e6 steps at CFL number 0.23 has 52.0 at the centre cells (written by\n")
        fh.write("# case_study_sigma.py from oracle.heat_spectral).\n")
        fh.write("# Columns: n mu steps amplitude sigma_cells closed_form_centre_at_steps\n")
        fh.write(f"{N} {MU} {STEPS} {AMP} {sigma} {f:.10f}\n")
    print(f"sigma {sigma}: centre {f:.10f}")


if __name__ == "__main__":
    main()
