"""Writes direct_hand.json: eq. (1) for three points in closed form.

Points (0,0,0), (1/2,0,0), (0,1/4,0) with potentials 1, -2, 1/2, so the
distances are r12 = 1/2, r13 = 1/4 and r23 = sqrt(5)/4.  Each kernel's three
sums are written out by hand below (singular kernels drop j = i, finite kernels
keep K(0)) and evaluated in 50-digit arithmetic (mpmath), then rounded to
double.  Nothing here calls the oracle or the library: these are the values the
oracle's direct sum is pinned to.  Run from the repository root:
    python tests/golden/make_direct_hand.py
"""
import json
import os

import mpmath as mp

mp.mp.dps = 50
HERE = os.path.dirname(os.path.abspath(__file__))

R12, R13, R23 = mp.mpf(1) / 2, mp.mpf(1) / 4, mp.sqrt(5) / 4
S = [mp.mpf(1), mp.mpf(-2), mp.mpf(1) / 2]


def sums(k, k0=None):
    """f_i = sum_j s_j k(r_ij); k0 = k(0) for a finite kernel, None drops j = i."""
    z = (lambda: 0) if k0 is None else (lambda: k0)
    return [S[0] * z() + S[1] * k(R12) + S[2] * k(R13),
            S[0] * k(R12) + S[1] * z() + S[2] * k(R23),
            S[0] * k(R13) + S[1] * k(R23) + S[2] * z()]


CASES = {
    "laplace": dict(param=0.0, k=lambda r: 1 / r, k0=None,
                    closed_form=["-2/(1/2) + (1/2)/(1/4) = -2",
                                 "1/(1/2) + (1/2)/sqrt(5/16) = 2 + sqrt(4/5)",
                                 "1/(1/4) - 2/sqrt(5/16) = 4 - 8/sqrt(5)"]),
    "sqdist": dict(param=0.0, k=lambda r: r * r, k0=mp.mpf(0),
                   closed_form=["-2/4 + 1/32 = -15/32", "1/4 + 5/32 = 13/32",
                                "1/16 - 5/8 = -9/16"]),
    "gauss": dict(param=0.01, k=lambda r: mp.exp(-r * r / mp.mpf("0.01")), k0=mp.mpf(1),
                  closed_form=["1 - 2 e^-25 + e^-6.25/2", "e^-25 - 2 + e^-31.25/2",
                               "e^-6.25 - 2 e^-31.25 + 1/2"]),
    "yukawa": dict(param=1.0, k=lambda r: mp.exp(-r) / r, k0=None,
                   closed_form=["-2 e^-1/2 / (1/2) + (1/2) e^-1/4 / (1/4)",
                                "e^-1/2/(1/2) + (1/2) e^-r23/r23",
                                "e^-1/4/(1/4) - 2 e^-r23/r23"]),
    # Sec. 5.4: cos(20 r)/r (singular) and sqrt(r^2 + 1) (finite, k(0) = 1)
    "cosr": dict(param=20.0, k=lambda r: mp.cos(20 * r) / r, k0=None,
                 closed_form=["-2 cos(10)/(1/2) + (1/2) cos(5)/(1/4) = -4 cos 10 + 2 cos 5",
                              "cos(10)/(1/2) + (1/2) cos(5 sqrt 5)/(sqrt(5)/4) = 2 cos 10 + (2/sqrt 5) cos(5 sqrt 5)",
                              "cos(5)/(1/4) - 2 cos(5 sqrt 5)/(sqrt(5)/4) = 4 cos 5 - (8/sqrt 5) cos(5 sqrt 5)"]),
    "mq": dict(param=1.0, k=lambda r: mp.sqrt(r * r + 1), k0=mp.mpf(1),
               closed_form=["1 - 2 sqrt(5/4) + (1/2) sqrt(17/16) = 1 - sqrt 5 + sqrt(17)/8",
                            "sqrt(5/4) - 2 + (1/2) sqrt(21/16) = sqrt(5)/2 - 2 + sqrt(21)/8",
                            "sqrt(17/16) - 2 sqrt(21/16) + 1/2 = sqrt(17)/4 - sqrt(21)/2 + 1/2"]),
}


def main():
    out = {
        "source": "eq. (1) of arXiv:1408.0210 evaluated in closed form for three points "
                  "(make_direct_hand.py, 50-digit arithmetic); singular kernels drop the "
                  "j=i term, finite kernels keep K(0)",
        "points": [[0.0, 0.0, 0.0], [0.5, 0.0, 0.0], [0.0, 0.25, 0.0]],
        "sigma": [1.0, -2.0, 0.5],
        "distances": {"r12": "1/2", "r13": "1/4", "r23": "sqrt(5/16)"},
        "expected": {},
    }
    for name, c in CASES.items():
        f = sums(c["k"], c["k0"])
        out["expected"][name] = {"param": c["param"], "f": [float(v) for v in f],
                                 "closed_form": c["closed_form"]}
    with open(os.path.join(HERE, "direct_hand.json"), "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    main()
