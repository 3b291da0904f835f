"""Writes the hand-worked fixtures of this folder from their closed forms (pure Python math; it calls
neither the oracle nor the HIP library).

residual_case.json -- one match of eq. (1), whitened and Huber-weighted as in Sec. III-A:
  T_i = identity; T_j = [2 I, (1, 0, 0)] (scale 2, no rotation). X_j = (0, 0, 3), X_i = (0, 0, 6).
  x = T_i^-1 T_j X_j = 2 (0, 0, 3) + (1, 0, 0) = (1, 0, 6), |x| = sqrt(37).
  e = (1/sqrt37, 0, 6/sqrt37 - 1, sqrt37 - 6).
  C_i = 4, C_j = 1 -> q = sqrt(4 * 1) = 2; r_c = sqrt(q) e_c / sigma_c, sigma = (0.003, 0.003, 0.003, 10).
  w_c = min(1, 1.345/|r_c|); rho(r) = r^2/2 (|r| <= 1.345), 1.345|r| - 1.345^2/2 otherwise.
"""
import json
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def residual_case():
    s37 = math.sqrt(37.0)
    e = [1.0 / s37, 0.0, 6.0 / s37 - 1.0, s37 - 6.0]
    q = math.sqrt(4.0 * 1.0)
    sig = [0.003, 0.003, 0.003, 10.0]
    k = 1.345
    r = [math.sqrt(q) * e[c] / sig[c] for c in range(4)]
    w = [1.0 if abs(x) <= k else k / abs(x) for x in r]
    E = sum(0.5 * x * x if abs(x) <= k else k * abs(x) - 0.5 * k * k for x in r)
    return {
        "cite": "eq. (1); whitening, Huber and IRLS weights of Sec. III-A; constants of Sec. IV-A",
        "pose_i": [0, 0, 0, 0, 0, 0, 1, 1.0],
        "pose_j": [1, 0, 0, 0, 0, 0, 1, 2.0],
        "X_i": [0, 0, 6.0], "X_j": [0, 0, 3.0], "C_i": 4.0, "C_j": 1.0,
        "e_expected": e, "r_expected": r, "w_expected": w, "E_expected": E,
    }


if __name__ == "__main__":
    with open(os.path.join(HERE, "residual_case.json"), "w") as f:
        json.dump(residual_case(), f, indent=1)
