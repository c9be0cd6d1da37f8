"""Writes the stored expected values under tests/golden from closed forms.

free_electron_tiny.json: V = 0 in the 10 bohr cube at Gamma, E_ref = 0.5 Ha.
The plane-wave energies are (1/2)(2 pi / 10)^2 |n|^2.  The eight states with
|n|^2 = 3 sit at 0.5922 Ha (distance 0.0922 from E); the next cluster is the
twelve |n|^2 = 2 states at 0.3948 Ha (distance 0.1052).
"""
import json
import math
import os

e1 = 0.5 * (2 * math.pi / 10.0) ** 2
out = {
    "eigenvalue": 3 * e1,
    "degeneracy": 8,
    "next_cluster": 2 * e1,
    "gap_to_next_cluster": abs(2 * e1 - 0.5) - abs(3 * e1 - 0.5),
    "source": "closed form (1/2)|2 pi n / L|^2, L = 10 bohr, n in {-1, 1}^3",
}
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "free_electron_tiny.json"), "w") as f:
    json.dump(out, f, indent=1)
    f.write("\n")
