"""Writes bernstein_degree10.json from exact rational closed forms of the
Bernstein basis (textbook identities, no oracle code)."""
import json
import os
from fractions import Fraction
from math import comb

N, TF = 10, 30


def main():
    half = [Fraction(comb(N, i), 2 ** N) for i in range(N + 1)]
    at0 = [Fraction(1 if i == 0 else 0) for i in range(N + 1)]
    at1 = [Fraction(1 if i == N else 0) for i in range(N + 1)]
    d0 = [Fraction(0)] * (N + 1)
    d0[0], d0[1] = Fraction(-N, TF), Fraction(N, TF)
    dd0 = [Fraction(0)] * (N + 1)
    k = Fraction(N * (N - 1), TF * TF)
    dd0[0], dd0[1], dd0[2] = k, -2 * k, k
    d1 = [Fraction(0)] * (N + 1)          # end slope: N (e_N - e_{N-1}) / tf
    d1[N - 1], d1[N] = Fraction(-N, TF), Fraction(N, TF)
    out = {
        "degree": N, "tf": TF,
        "P_tau0": [str(v) for v in at0], "P_tau_half": [str(v) for v in half],
        "P_tau1": [str(v) for v in at1], "Pd_tau0": [str(v) for v in d0],
        "Pd_tau1": [str(v) for v in d1], "Pdd_tau0": [str(v) for v in dd0],
    }
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "bernstein_degree10.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
