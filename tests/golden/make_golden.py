"""Writes the oracle regression fixtures in this folder.

The paper prints no worked numeric example (its only numbers are timings), so
these fixtures are not the paper's values: they freeze the FP64 oracle's
output on two tiny seeded inputs, one per regularisation form, so that a
later change to the oracle's arithmetic shows up as a diff.  Only ``oracle/``
is called.  Run from the repository root:  python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import hgf_oracle as O  # noqa: E402


def tiny_inputs():
    rng = np.random.default_rng(20180301)
    I = rng.uniform(0, 1, size=(3, 9, 11))
    V = rng.uniform(0, 0.5, size=(9, 11, 3))
    return I, V


def cases():
    I, V = tiny_inputs()
    # covariance form, full monomial basis of degree 2 (n = 9), r = 2, eps = 1e-3
    yield "covariance_monomial_d2_r2.txt", O.filter_covariance(O.guidance(I, 2, "monomial"), V, 2, 1e-3)
    # ridge form with the paper's experimental parameters: lambda = 0.05, power basis
    # G_{(i-1)d+j} = I_i^j with d = 2 (Sec. 6), here with r = 3 on the tiny image
    yield "ridge_power_d2_r3.txt", O.filter_ridge(O.guidance(I, 2, "power"), V, 3, 0.05)


def main():
    for name, Z in cases():
        np.savetxt(os.path.join(HERE, name), Z.reshape(-1, Z.shape[-1]), fmt="%.17e")


if __name__ == "__main__":
    main()
